"""Host checks of the arithmetic the kernels use for a particle's home cell:
division by the lattice side through a multiply and shift, and the lattice
offset (2 rem - np) / (2 np) as a double product rounded once to float.
Both must equal the plain integer division and the correctly rounded float32
quotient for every lattice side 1 .. 1024, so the home cells stay the ones
the FP32 replay in oracle/cic_fp32.py computes."""
import numpy as np
import pytest


def magic(d):
    l = 0
    while (1 << l) < d:
        l += 1
    s = 30 + l
    return ((1 << s) + d - 1) // d, s


@pytest.mark.parametrize("lo,hi", [(1, 256), (256, 512), (512, 769), (769, 1025)])
def test_multiply_shift_division_is_exact(lo, hi):
    rng = np.random.default_rng(lo)
    for d in range(lo, hi):
        m, s = magic(d)
        assert m < 2 ** 32
        n = np.concatenate([
            rng.integers(0, 2 ** 30, 4000, dtype=np.uint64),
            np.arange(0, 4 * d, dtype=np.uint64),
            (np.arange(1, 2000, dtype=np.uint64) * d) - 1,
            np.array([2 ** 30 - 1, (2 ** 30 - 1) // d * d, (2 ** 30 - 1) // d * d - 1], dtype=np.uint64),
        ])
        n = n[n < 2 ** 30]
        q = (n.astype(object) * m) >> s
        assert np.array_equal(np.array(q, dtype=np.uint64), n // np.uint64(d)), d


def test_multiply_shift_division_exhaustive_for_the_largest_sides():
    # every n below 2^30 (n m < 2^62 fits in 64 bits) for two sides whose
    # magic numbers carry the most rounding
    for d in (1023, 769):
        m, s = magic(d)
        for base in range(0, 2 ** 30, 2 ** 24):
            n = np.arange(base, base + 2 ** 24, dtype=np.uint64)
            q = (n * np.uint64(m)) >> np.uint64(s)
            assert np.array_equal(q, n // np.uint64(d)), (d, base)


def test_lattice_offset_double_product_equals_float_quotient():
    for d in range(1, 1025):
        a = np.arange(-d, d, dtype=np.int64)
        want = a.astype(np.float32) / np.float32(2 * d)
        got = (a.astype(np.float64) * (1.0 / (2.0 * d))).astype(np.float32)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), d
