"""Pins for the float32 replay of the fixed-point CIC mass deposit."""
import itertools
from fractions import Fraction

import numpy as np

from oracle import cic_fp32, pm

F32 = np.float32


def random_disp(np_side, nm, scale, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((3, np_side ** 3)) * scale).astype(F32)


def test_replay_matches_fp64_deposit():
    np_side, nm, L = 8, 16, 20.0
    disp = random_disp(np_side, nm, 3.0, 0)
    from oracle.ic import lattice
    pos = lattice(np_side, L) + disp.astype(np.float64) * (L / nm)
    ref = pm.cic_deposit(pos, nm, L)
    rho = cic_fp32.density(disp, np_side, nm, contrast=False)
    assert np.abs(rho - ref).max() < 2e-6 * ref.max()
    assert abs(float(rho.astype(np.float64).sum()) - np_side ** 3) < 1e-5 * np_side ** 3


def _round_to_f32(x: Fraction) -> np.float32:
    """Correctly rounded (to nearest, ties to even) float32 of a non-negative rational."""
    if x == 0:
        return F32(0.0)
    e = x.numerator.bit_length() - x.denominator.bit_length()
    if Fraction(2) ** e > x:
        e -= 1
    scaled = x / Fraction(2) ** (e - 23)             # in [2^23, 2^24)
    m = scaled.numerator // scaled.denominator
    rest = scaled - m
    if rest > Fraction(1, 2) or (rest == Fraction(1, 2) and m % 2 == 1):
        m += 1
    return F32(float(Fraction(m) * Fraction(2) ** (e - 23)))


def test_node_mass_is_the_correctly_rounded_exact_sum_of_the_weights():
    # With every float32 weight >= 2^-9 (fractions kept in [0.15, 0.85]) the
    # node mass is the exact rational sum of its float32 weights, rounded
    # once to float32 -- whatever order the particles come in.
    np_side, nm = 4, 8
    rng = np.random.default_rng(1)
    base = cic_fp32._axis_terms(np_side, nm)[1][0]          # -1/2 on a 2x mesh
    lat = np.stack(np.meshgrid(*([np.arange(np_side)] * 3), indexing="ij")).reshape(3, -1) * (nm // np_side)
    target = rng.integers(0, nm, (3, np_side ** 3)) + rng.uniform(0.15, 0.85, (3, np_side ** 3))
    target[:, 5:12] = target[:, 4:5]                          # several particles in one cell
    target[:, 6] += 1e-3
    disp = (target - lat - base).astype(F32)
    cells, f = cic_fp32.home_cells(disp, np_side, nm)
    assert f.min() > 0.1 and f.max() < 0.9
    w = cic_fp32.weights(f)
    assert w.min() >= 2.0 ** -9
    exact = {}
    for p in range(np_side ** 3):
        for k in range(8):
            s = ((k >> 2) & 1, (k >> 1) & 1, k & 1)
            n = tuple(int((cells[e, p] + s[e]) % nm) for e in range(3))
            exact[n] = exact.get(n, Fraction(0)) + Fraction(float(w[k, p]))
    rho = cic_fp32.density(disp, np_side, nm, contrast=False)
    for n in itertools.product(range(nm), repeat=3):
        want = _round_to_f32(exact.get(n, Fraction(0)))
        assert want.tobytes() == rho[n].tobytes(), n


def test_fixed_point_weights_round_to_nearest_even():
    w = np.array([1.0, 0.5, 2.0 ** -9, 2.0 ** -33, 3 * 2.0 ** -33, 2.0 ** -34, 0.0], dtype=F32)
    q = cic_fp32.fixed_point(w)
    assert q.tolist() == [2 ** 32, 2 ** 31, 2 ** 23, 0, 2, 0, 0]


def test_node_sampled_replay_equals_full_replay():
    np_side, nm = 8, 16
    disp = random_disp(np_side, nm, 2.0, 2)
    full = cic_fp32.density(disp, np_side, nm)
    nodes = np.random.default_rng(3).integers(0, nm, (40, 3))
    part = cic_fp32.density_at_nodes(disp, np_side, nm, nodes)
    assert full[tuple(nodes.T)].tobytes() == part.tobytes()


def test_lattice_home_cells_are_cell_centred():
    # Zero displacement: lattice points sit half a cell above a node.
    cells, f = cic_fp32.home_cells(np.zeros((3, 4 ** 3), F32), 4, 12)
    assert np.all(f == F32(0.5))
    assert set(np.unique(cells[0])) == {0 + 2, 3 + 2, 6 + 2, 9 + 2}


def test_chunked_node_replay_equals_full_replay():
    # the chunked scan (used where all particles' temporaries do not fit in
    # host memory) keeps exactly the feeding particles, in ascending id
    rng = np.random.default_rng(12)
    n, nm = 16, 32
    disp = (rng.standard_normal((3, n ** 3)) * 2.0).astype(np.float32)
    disp[:, :500] = (np.float32(7.3) - cic_fp32._axis_terms(n, nm)[0][0]).astype(np.float32)  # a crowded cell
    nodes = np.r_[rng.integers(0, nm, (40, 3)), [[7, 7, 7], [8, 8, 8], [0, 0, 0], [31, 31, 31]]]
    full = cic_fp32.density_at_nodes(disp, n, nm, nodes)
    seen = []
    for chunk in (777, 4096, n ** 3):
        got = cic_fp32.density_at_nodes_chunked(disp, n, nm, nodes, chunk=chunk,
                                                progress=lambda a, b: seen.append((a, b)))
        assert got.tobytes() == full.tobytes()
    assert seen[-1] == (n ** 3, n ** 3)
