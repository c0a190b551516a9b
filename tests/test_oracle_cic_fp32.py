"""Pins for the float32 same-order CIC replay."""
import itertools

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


def test_replay_against_scalar_loop():
    # Literal scalar float32 loop over nodes, offsets and particles.
    np_side, nm = 4, 8
    disp = random_disp(np_side, nm, 1.5, 1)
    disp[:, 5] = disp[:, 9]                     # several particles in one cell
    disp[:, 6] = disp[:, 9] + F32(1e-3)
    rho = cic_fp32.density(disp, np_side, nm, contrast=False)
    cells, f = cic_fp32.home_cells(disp, np_side, nm)
    for n in itertools.product(range(nm), repeat=3):
        acc = F32(0.0)
        for k in range(7, -1, -1):           # source cells in ascending index
            s = ((k >> 2) & 1, (k >> 1) & 1, k & 1)
            c = [(n[e] - s[e]) % nm for e in range(3)]
            part = F32(0.0)
            for p in range(np_side ** 3):
                if all(cells[e, p] == c[e] for e in range(3)):
                    w = [[F32(1.0) - f[e, p], f[e, p]] for e in range(3)]
                    part = F32(part + F32(F32(w[0][s[0]] * w[1][s[1]]) * w[2][s[2]]))
            acc = F32(acc + part)
        assert acc.tobytes() == rho[n].tobytes(), n


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
