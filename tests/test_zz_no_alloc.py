"""cola_density_noalloc (the allocation-free density entry point with its
sort buffers in a static device array) against cola_density_of through the
C ABI: bitwise equal on two calls in a row, the second smaller than the
first, and the FP32 same-order replay of the oracle."""
import ctypes as C

import numpy as np
import pytest

from _progress import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import cic_fp32  # noqa: E402
from paper_1507_05329_amd import _lib  # noqa: E402


def noalloc_density(disp, np_side, nm):
    lib = _lib.load()
    out = torch.empty((nm,) * 3, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    r = lib.cola_density_noalloc(C.c_void_p(disp.data_ptr()), np_side, nm, C.c_void_p(out.data_ptr()),
                                 C.c_void_p(stream))
    assert r == _lib.COLA_OK, r
    return out


def context_density(disp, np_side, nm):
    from paper_1507_05329_amd.sim import ColaSim
    s = ColaSim(np_side, nm, 100.0)
    try:
        return s.density(disp=disp)
    finally:
        s.close()


def clustered(np_side, nm, seed):
    rng = np.random.default_rng(seed)
    q = np.stack(np.meshgrid(*([np.arange(np_side) * (nm / np_side)] * 3), indexing="ij")).reshape(3, -1)
    target = q + rng.standard_normal(q.shape) * 1.5
    target[:, :500] = nm * 0.3 + rng.uniform(0, 1, (3, 500))        # a dense clump in one cell
    return (target - q).astype(np.float32)


def test_noalloc_density_equals_context_density_twice():
    for np_side, nm, seed in ((64, 256, 1), (32, 64, 2)):          # the second call is smaller
        say(f"[gpu] noalloc density {np_side}^3 / {nm}^3")
        d = torch.from_numpy(clustered(np_side, nm, seed)).cuda()
        got = noalloc_density(d, np_side, nm)
        want = context_density(d, np_side, nm)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        ref = cic_fp32.density(d.cpu().numpy(), np_side, nm)
        assert got.cpu().numpy().tobytes() == ref.tobytes()


def test_noalloc_density_rejects_sizes_beyond_its_array():
    lib = _lib.load()
    d = torch.zeros(3 * 80 ** 3, dtype=torch.float32, device="cuda")
    out = torch.empty(512 ** 3 // 8, dtype=torch.float32, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.cola_density_noalloc(C.c_void_p(d.data_ptr()), 80, 96, C.c_void_p(out.data_ptr()), s) \
        == _lib.COLA_ENOMEM                                           # 80^3 particles > 64^3
    assert lib.cola_density_noalloc(C.c_void_p(d.data_ptr()), 32, 512, C.c_void_p(out.data_ptr()), s) \
        == _lib.COLA_ENOMEM                                           # 512^3 mesh > 256^3
    assert lib.cola_density_noalloc(C.c_void_p(d.data_ptr()), 40, 64, C.c_void_p(out.data_ptr()), s) \
        == _lib.COLA_EINVAL                                           # np not a multiple of 16
