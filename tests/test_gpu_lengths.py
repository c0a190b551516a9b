"""Every compiled transform length, element by element, through the C ABI.

* cola_fft3d forward and inverse at 16 ... 768 against FP64 rfftn.
* cola_pm_gradient (r2c FFT, Green's function x ik fused in the x pass, the
  inverse y passes, the c2r pass: the step's spectral pipeline) at every
  mesh length 32 ... 768 against the oracle's force meshes of the same
  density field.
* 1024, 1536, 2048 (too big for the FP64 oracle on the host): a sum of 8
  plane waves with seeded amplitudes and phases, whose spectrum and force
  meshes are known in closed form (Green's function of a single mode:
  g_d = -alpha n_d / (2 pi |n|^2) A sin(theta) in mesh units), checked at
  every element on the device; at 2048 also a seeded white field against
  the FP64 oracle at 24 sampled nodes (the oracle sums the inverse
  transform mode by mode there).
"""
import math

import numpy as np
import pytest

from _progress import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import cosmology as cosmo, pm  # noqa: E402

BOX = 100.0
OM = 0.27


def padded_cols(n):
    return ((n // 2 + 1) + 15) // 16 * 16


def rel_l2(a, b):
    a = np.asarray(a)
    a = a.astype(np.complex128) if np.iscomplexobj(a) else a.astype(np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def context(n):
    from paper_1507_05329_amd.sim import ColaSim
    return ColaSim(16, max(n, 32), BOX)


@pytest.mark.parametrize("n", [16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768])
def test_fft3d_every_length_against_rfftn(n):
    import scipy.fft as sfft
    say(f"[gpu] fft3d n={n} against FP64 rfftn")
    s = context(n)
    try:
        x = np.random.default_rng(n).standard_normal((n, n, n)).astype(np.float32)
        m = np.zeros((n, n, 2 * padded_cols(n)), np.float32)
        m[:, :, :n] = x
        t = torch.from_numpy(m).cuda()
        del m
        s.fft3d(t, n)
        got = t.cpu().numpy().view(np.complex64)[:, :, : n // 2 + 1]
        ref = sfft.rfftn(x.astype(np.float64), workers=-1)
        err = rel_l2(got, ref)
        del got, ref
        s.fft3d(t, n, inverse=True)
        back = t.cpu().numpy()[:, :, :n] / float(n) ** 3
        err_inv = rel_l2(back, x)
        say(f"[gpu]   forward rel-L2 {err:.2e}, round trip {err_inv:.2e}")
        assert err < 2e-6 and err_inv < 2e-6
    finally:
        s.close()


@pytest.mark.parametrize("n", [32, 48, 64, 96, 128, 192, 256, 384, 512, 768])
def test_pm_gradient_every_mesh_length_against_oracle(n):
    import scipy.fft as sfft
    say(f"[gpu] pm_gradient n={n} against the oracle's force meshes")
    s = context(n)
    try:
        a = 0.5
        alpha = cosmo.poisson_alpha(a, OM)
        delta = np.random.default_rng(100 + n).standard_normal((n, n, n)).astype(np.float32)
        g = s.pm_gradient(a, torch.from_numpy(delta).cuda())
        dk = sfft.rfftn(delta.astype(np.float64), workers=-1)
        for d in range(3):
            ref = pm.force_component(dk, n, BOX, alpha, d) * (n / BOX)
            err = rel_l2(g[d].cpu().numpy(), ref)
            say(f"[gpu]   g_{d} rel-L2 {err:.2e}")
            assert err <= 1e-5
    finally:
        s.close()


# ---------------------------------------------------------------------------
# Plane waves at the lengths the FP64 oracle cannot hold.

def plane_waves(n, seed, nw=8):
    """nw distinct modes (no pair v, -v; every |v_e| < n/2, so no Nyquist
    plane), amplitudes in [0.5, 2], phases in [0, 2 pi)."""
    rng = np.random.default_rng(seed)
    # one low mode and one near the Nyquist corner, then random ones
    modes = [(1, 0, 2), (n // 2 - 1, -(n // 2 - 2), n // 2 - 1)]
    while len(modes) < nw:
        v = tuple(int(x) for x in rng.integers(-n // 2 + 1, n // 2, 3))
        if v == (0, 0, 0) or v in modes or tuple(-x for x in v) in modes:
            continue
        modes.append(v)
    return [(v, float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.0, 2 * math.pi))) for v in modes]


class WaveField:
    """sum_w A_w f(theta_w(i, j, k)), theta = 2 pi (v . (i, j, k)) / n + phi,
    evaluated in float64 on the device, a block of x planes at a time."""

    def __init__(self, waves, n, dev):
        self.waves, self.n, self.dev = waves, n, dev
        j = torch.arange(n, dtype=torch.int64, device=dev)
        self.cs = []
        for v, _, _ in waves:
            jk = (v[1] * j[:, None] + v[2] * j[None, :]) % n           # exact integer phase
            b = jk.to(torch.float64) * (2 * math.pi / n)
            self.cs.append((torch.cos(b), torch.sin(b)))

    def block(self, i0, i1, weights, use_sin):
        n = self.n
        ii = torch.arange(i0, i1, dtype=torch.int64, device=self.dev)
        out = torch.zeros((i1 - i0, n, n), dtype=torch.float64, device=self.dev)
        for (v, amp, phi), (c, s), wt in zip(self.waves, self.cs, weights):
            if wt == 0.0:
                continue
            a = ((v[0] * ii) % n).to(torch.float64) * (2 * math.pi / n) + phi
            ca, sa = torch.cos(a)[:, None, None], torch.sin(a)[:, None, None]
            if use_sin:                                   # sin(a + b) = sin a cos b + cos a sin b
                out += (amp * wt) * (sa * c[None] + ca * s[None])
            else:                                         # cos(a + b) = cos a cos b - sin a sin b
                out += (amp * wt) * (ca * c[None] - sa * s[None])
        return out


def chunk_planes(n):
    return max(1, (1 << 27) // (n * n))                  # 1 GiB of float64 per block


@pytest.mark.timeout(900)
@pytest.mark.parametrize("n", [1024, 1536, 2048])
def test_large_lengths_plane_waves(n):
    from paper_1507_05329_amd.sim import ColaSim
    dev = torch.device("cuda:0")
    waves = plane_waves(n, seed=n)
    say(f"[gpu] plane waves n={n}: {[w[0] for w in waves]}")
    s = ColaSim(16, n, BOX)
    try:
        wf = WaveField(waves, n, dev)
        ones = [1.0] * len(waves)
        cp = chunk_planes(n)
        P = padded_cols(n)
        # -- forward r2c FFT: spikes of height A n^3 / 2 at +-v, zero elsewhere
        mesh = torch.zeros((n, n, 2 * P), dtype=torch.float32, device=dev)
        for i0 in range(0, n, cp):
            i1 = min(n, i0 + cp)
            mesh[i0:i1, :, :n] = wf.block(i0, i1, ones, use_sin=False).to(torch.float32)
        s.fft3d(mesh, n)
        spec = mesh.view(torch.complex64)                 # (n, n, P)
        expect = {}
        for (v, amp, phi) in waves:
            val = 0.5 * amp * float(n) ** 3 * complex(math.cos(phi), math.sin(phi))
            if v[2] >= 0:
                key = (v[0] % n, v[1] % n, v[2])
                expect[key] = expect.get(key, 0) + val
            if v[2] <= 0:
                key = ((-v[0]) % n, (-v[1]) % n, -v[2])
                expect[key] = expect.get(key, 0) + val.conjugate()
        got = {key: complex(spec[key].item()) for key in expect}
        spike_err = sum(abs(got[k] - expect[k]) ** 2 for k in expect)
        ref2 = sum(abs(x) ** 2 for x in expect.values())
        for key in expect:
            spec[key] = 0
        rest = 0.0
        half = n // 2 + 1
        for i0 in range(0, n, cp):
            blk = torch.view_as_real(spec[i0:min(n, i0 + cp), :, :half]).to(torch.float64)
            rest += float((blk * blk).sum())
            del blk
        err = math.sqrt((spike_err + rest) / ref2)
        say(f"[gpu]   forward rel-L2 {err:.2e} (spikes {math.sqrt(spike_err / ref2):.2e})")
        assert err < 2e-6
        for key, val in got.items():
            spec[key] = val
        # -- inverse (c2r): back to n^3 times the input
        s.fft3d(mesh, n, inverse=True)
        num = den = 0.0
        for i0 in range(0, n, cp):
            i1 = min(n, i0 + cp)
            ref = wf.block(i0, i1, ones, use_sin=False)
            d = mesh[i0:i1, :, :n].to(torch.float64) / float(n) ** 3 - ref
            num += float((d * d).sum())
            den += float((ref * ref).sum())
            del d, ref
        err_inv = math.sqrt(num / den)
        say(f"[gpu]   round trip rel-L2 {err_inv:.2e}")
        assert err_inv < 2e-6
        del mesh, spec
        torch.cuda.empty_cache()
        # -- force meshes of delta = the same waves
        a = 0.5
        alpha = cosmo.poisson_alpha(a, OM)
        delta = torch.empty((n, n, n), dtype=torch.float32, device=dev)
        for i0 in range(0, n, cp):
            i1 = min(n, i0 + cp)
            delta[i0:i1] = wf.block(i0, i1, ones, use_sin=False).to(torch.float32)
        for d in range(3):
            g = s.pm_gradient(a, delta, comps=(d,))[d]
            # g_d = sum_w -A_w alpha n / (2 pi) * v_d / |v|^2 * sin(theta_w)
            wts = [-alpha * n / (2 * math.pi) * v[d] / float(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
                   for v, _, _ in waves]
            num = den = 0.0
            for i0 in range(0, n, cp):
                i1 = min(n, i0 + cp)
                ref = wf.block(i0, i1, wts, use_sin=True)
                dd = g[i0:i1].to(torch.float64) - ref
                num += float((dd * dd).sum())
                den += float((ref * ref).sum())
                del dd, ref
            del g
            torch.cuda.empty_cache()
            err = math.sqrt(num / den)
            say(f"[gpu]   g_{d} rel-L2 {err:.2e}")
            assert err <= 1e-5
    finally:
        s.close()
        torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# A seeded white field on the 2048 mesh (the kernels, launch shapes and
# schedules of the 1024^3/2048^3 step) against the FP64 oracle at sampled
# nodes: the oracle transforms the field slab by slab and sums the inverse
# transform mode by mode at each node (oracle/pm.py: rfftn_slabs,
# force_at_nodes), within the host memory of one command.

def white_field(n, seed, threads=16):
    """Uniform in [-1, 1), float32; one generator per 8 x planes, spawned from
    the seed, filled in parallel."""
    from concurrent.futures import ThreadPoolExecutor
    seeds = np.random.SeedSequence(seed).spawn(n // 8)
    out = np.empty((n, n, n), np.float32)

    def fill(i):
        blk = out[8 * i:8 * (i + 1)]
        np.random.default_rng(seeds[i]).random(out=blk, dtype=np.float32)
        blk *= 2.0
        blk -= 1.0

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(fill, range(n // 8)))
    return out


def reporter(tag):
    seen = set()

    def cb(what, done, total):
        q = (4 * done) // total
        if (what, q) not in seen:
            seen.add((what, q))
            say(f"[gpu]   {tag}: {what} {min(done, total)}/{total}")
    return cb


@pytest.mark.timeout(1500)
def test_pm_gradient_2048_random_field_at_sampled_nodes():
    from paper_1507_05329_amd.sim import ColaSim
    n, a = 2048, 0.5
    alpha = cosmo.poisson_alpha(a, OM)
    say("[gpu] pm_gradient n=2048 on a seeded white field: generating it")
    delta = white_field(n, 2048)
    rng = np.random.default_rng(7)
    nodes = np.concatenate([[[0, 0, 0], [n - 1, n - 1, n - 1], [n // 2, n // 2, n // 2], [1, n - 2, n // 2 + 1]],
                            rng.integers(0, n, (20, 3))]).astype(np.int64)
    got = np.empty((3, len(nodes)))
    s = ColaSim(16, n, BOX)
    try:
        dev = torch.from_numpy(delta).cuda()
        ix = [torch.from_numpy(nodes[:, e]).cuda() for e in range(3)]
        for d in range(3):
            g = s.pm_gradient(a, dev, comps=(d,))[d]
            got[d] = g[ix[0], ix[1], ix[2]].cpu().numpy()
            del g
        del dev
        say("[gpu]   device force meshes sampled")
    finally:
        s.close()
        torch.cuda.empty_cache()
    dk = pm.rfftn_slabs(delta, slab=64, progress=reporter("oracle FP64 transform"))
    del delta
    ref, rms = pm.force_at_nodes(dk, n, BOX, alpha, nodes, slab=16, progress=reporter("oracle mode sums"))
    del dk
    ref *= n / BOX
    rms *= n / BOX
    for d in range(3):
        worst = float(np.abs(got[d] - ref[d]).max() / rms[d])
        rel = float(np.linalg.norm(got[d] - ref[d]) / np.linalg.norm(ref[d]))
        say(f"[gpu]   g_{d}: max |diff| / rms {worst:.2e}, rel-L2 over the nodes {rel:.2e}")
        assert worst <= 1e-5 and rel <= 1e-5
