"""The FFT schedule table and its autotuner: every column-pass block order
gives the same force field bit for bit (the order decides which workgroup
transforms which column, not the arithmetic), and the autotuner keeps one
of its candidates."""
import itertools

import pytest

from _progress import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _order_mismatches(s, n, kinds):
    """Every combination of block orders against the first; returns what
    differed.  The device tensors live only in this frame, so a failing
    assertion in the caller keeps none of them alive."""
    from paper_1507_05329_amd import _lib
    from paper_1507_05329_amd.sim import fft_schedule
    bad = []
    delta = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(n)
    delta.normal_(generator=gen)
    comps = (0, 1, 2) if n < 2048 else (1,)
    ref = None
    for orders in itertools.product((1, 0), repeat=3):
        for k, o in zip(kinds, orders):
            fft_schedule(n, k, o)
        g = s.pm_gradient(0.5, delta, comps=comps)
        if ref is None:
            ref = {d: g[d].clone() for d in comps}
        else:
            bad += [("pm_gradient", orders, d) for d in comps if not torch.equal(g[d], ref[d])]
        del g
    del ref
    torch.cuda.empty_cache()
    # the plain passes of cola_fft3d too (memory allows it below 2048)
    if n < 2048:
        m = torch.zeros((n, n, 2 * (((n // 2 + 1) + 15) // 16 * 16)), dtype=torch.float32, device="cuda")
        m[:, :, :n] = delta
        outs = []
        for o in (1, 0):
            fft_schedule(n, _lib.PASS_PLAIN, o)
            t = m.clone()
            s.fft3d(t, n)
            outs.append(t)
        if not torch.equal(outs[0], outs[1]):
            bad.append(("fft3d", o))
    return bad


@pytest.mark.parametrize("n", [64, 192, 768, 2048])
def test_column_pass_block_orders_give_identical_forces(n):
    from paper_1507_05329_amd import _lib
    from paper_1507_05329_amd.sim import ColaSim, fft_schedule
    say(f"[gpu] column-pass block orders at n={n}")
    kinds = (_lib.PASS_PLAIN, _lib.PASS_GREEN, _lib.PASS_GRAD)
    s = ColaSim(16, n, 100.0)
    before = [fft_schedule(n, k) for k in kinds]
    try:
        bad = _order_mismatches(s, n, kinds)
        torch.cuda.empty_cache()
        assert not bad, bad
        best, ms = s.autotune(reps=2)
        say(f"[gpu]   autotune: {best}, ms {ms}")
        assert set(best.values()) <= {0, 1}
        assert [fft_schedule(n, k) for k in kinds] == [best["plain"], best["green"], best["grad"]]
        assert all(v > 0 for v in ms.values())
    finally:
        for k, b in zip(kinds, before):
            fft_schedule(n, k, b)
        s.close()
        torch.cuda.empty_cache()
