"""Pins for the oracle's friends-of-friends groups (Sec. 2.3, Sec. 3.1: b = 0.2)."""
import numpy as np
import pytest

from oracle import fof


def clustered_disp(np_side, nm, seed, spread=0.6):
    # particles pulled towards a few centres: groups of many sizes
    rng = np.random.default_rng(seed)
    q = fof.lattice_fp32(np_side, nm).astype(np.float64)
    centres = rng.uniform(0, nm, (3, 4))
    pick = rng.integers(0, 4, q.shape[1])
    target = centres[:, pick] + rng.normal(0, spread * nm / np_side, q.shape)
    pull = rng.uniform(0.3, 1.0, q.shape[1])
    return ((target - q) * pull).astype(np.float32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tree_equals_brute_force(seed):
    d = clustered_disp(8, 16, seed)
    a = fof.fof_labels(d, 8, 16)
    b = fof.fof_labels_brute(d, 8, 16)
    assert np.array_equal(a, b)
    assert len(np.unique(a)) < len(a)            # some groups formed
    assert (np.bincount(a) > 1).sum() > 3


def single_pair(dz, b_frac):
    # np = 4 on an 8-mesh: spacing 2 cells; particle 1 sits at lattice (0, 0, 2)
    d = np.zeros((3, 64), np.float32)
    d[2, 1] = np.float32(dz)
    return fof.fof_labels_brute(d, 4, 8, b_frac), fof.fof_labels(d, 4, 8, b_frac)


def test_link_decision_at_the_linking_length():
    # b_frac = 0.125: b = 0.25 cells, b^2 = 0.0625 exactly; separation 0.25 links, 0.26 does not
    for lab in single_pair(-1.75, 0.125):
        assert lab[1] == 0 and (lab[2:] == np.arange(2, 64)).all()
    for lab in single_pair(-1.74, 0.125):
        assert (lab == np.arange(64)).all()


def test_nearest_image_across_the_box_edge():
    d = np.zeros((3, 64), np.float32)
    d[2, 0] = np.float32(-0.1)          # x = -0.1, i.e. 7.9 in the box
    d[2, 3] = np.float32(1.95)          # lattice z = 6: x = 7.95, 0.05 from particle 0 through the edge
    d[2, 1] = np.float32(-1.82)         # lattice z = 2: x = 0.18, 0.28 from particle 0
    for lab in (fof.fof_labels_brute(d, 4, 8, 0.15), fof.fof_labels(d, 4, 8, 0.15)):   # b = 0.3
        assert lab[0] == lab[1] == lab[3] == 0
        assert lab[2] == 2


def test_chain_is_one_group_labelled_by_its_smallest_id():
    # particles 5, 21, 37, 53 (lattice x = 0..3, y = 1, z = 1) pulled onto a line 0.9 b apart
    np_side, nm, b_frac = 4, 8, 0.2                   # b = 0.4 cells
    d = np.zeros((3, 64), np.float32)
    ids = [53, 37, 21, 5]
    for k, i in enumerate(ids):
        ix = i // 16
        d[0, i] = np.float32(3.0 + 0.36 * k - 2.0 * ix)
    for lab in (fof.fof_labels_brute(d, np_side, nm, b_frac), fof.fof_labels(d, np_side, nm, b_frac)):
        assert (lab[ids] == 5).all()
        others = np.setdiff1d(np.arange(64), ids)
        assert (lab[others] == others).all()


@pytest.mark.parametrize("seed", [3, 4])
def test_labels_are_smallest_ids_of_their_groups(seed):
    d = clustered_disp(8, 16, seed)
    lab = fof.fof_labels(d, 8, 16)
    ids = np.arange(len(lab))
    assert (lab <= ids).all()
    assert (lab[lab] == lab).all()
    # every friend pair shares a label, and a label's group holds its own id
    x = fof.positions_fp32(d, 8, 16)
    a, b = np.triu_indices(len(lab), 1)
    friends = fof.r2_fp32(x, a, b, 16) <= fof.link_length_sq(0.2, 8, 16)
    assert (lab[a[friends]] == lab[b[friends]]).all()


def test_halo_catalogue_straddling_the_edge_and_counts():
    # a chain across the box edge: the centre is the mean of the unwrapped members
    d = np.zeros((3, 64), np.float32)
    d[2, 0] = np.float32(-0.1)           # x = -0.1
    d[2, 3] = np.float32(1.95)           # x = 7.95
    d[2, 1] = np.float32(-1.82)          # x = 0.18
    vel = np.zeros((3, 64), np.float32)
    vel[0, [0, 1, 3]] = [1.0, 2.0, 6.0]
    lab = fof.fof_labels(d, 4, 8, 0.15)
    roots, counts, com, vm = fof.halo_catalogue(d, vel, lab, 4, 8, 2)
    assert roots.tolist() == [0] and counts.tolist() == [3]
    want_z = np.mod((-0.1 + 0.18 - 0.05) / 3.0, 8)      # members at -0.1, 0.18, -0.05
    assert com[2, 0] == pytest.approx(want_z, abs=1e-6)
    assert com[0, 0] == pytest.approx(0.0, abs=1e-12) and com[1, 0] == pytest.approx(0.0, abs=1e-12)
    assert vm[0, 0] == pytest.approx(3.0)
    # every group of the clustered case is listed once with its size
    d = clustered_disp(8, 16, 5)
    lab = fof.fof_labels(d, 8, 16)
    roots, counts, _, _ = fof.halo_catalogue(d, None, lab, 8, 16, 1)
    assert counts.sum() == lab.size and (lab[roots] == roots).all()
