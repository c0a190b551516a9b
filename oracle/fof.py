"""Friends-of-friends groups of the particles (Koda et al. 2015: the halo
finder run on the fly in Sec. 2.3, linking length 0.2 times the mean particle
separation in Sec. 3.1), as a plain reference.

Test infrastructure: the slow, plainly written reference that the GPU path is
checked against; nothing in the library imports it.

Two particles are friends when their periodic separation is at most the
linking length b; groups are the connected components of that relation.  A
group is labelled by its smallest particle id, so the labels are unique.

The decision "separation <= b" is taken in float32, in the same order of
operations as the GPU (where floating point decides an integer, both sides
decide in the same precision), on the state's float32 displacement in mesh
units:
    q_e  = float32(i_e * nm) / float32(np)           (lattice point, mesh units)
    x_e  = q_e + d_e
    dx_e = x_e(a) - x_e(b);  dx_e -= nm * rint(dx_e / nm)   (nearest image)
    r2   = (dx_0^2 + dx_1^2) + dx_2^2,   friends iff r2 <= float32(b^2)
each step one correctly rounded float32 operation.  Candidate pairs come from
a float64 k-d tree with a slightly larger radius; the float32 test decides.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

F32 = np.float32


def lattice_fp32(np_side: int, nm: int) -> np.ndarray:
    """(3, np^3) float32 lattice points in mesh units, C order of the ids."""
    i = np.arange(np_side, dtype=np.int64)
    q1 = (i * nm).astype(F32) / F32(np_side)
    g = np.meshgrid(q1, q1, q1, indexing="ij")
    return np.stack([a.reshape(-1) for a in g])


def positions_fp32(disp: np.ndarray, np_side: int, nm: int) -> np.ndarray:
    return lattice_fp32(np_side, nm) + disp.astype(F32)


def r2_fp32(x: np.ndarray, a: np.ndarray, b: np.ndarray, nm: int) -> np.ndarray:
    """Squared nearest-image separation of the pairs (a, b), float32."""
    nmf = F32(nm)
    r2 = None
    for e in range(3):
        dx = x[e, a] - x[e, b]
        dx = dx - nmf * np.rint(dx / nmf)
        t = dx * dx
        r2 = t if r2 is None else r2 + t
    return r2


def link_length_sq(b_frac: float, np_side: int, nm: int) -> np.float32:
    b = b_frac * nm / np_side
    return F32(b * b)


def candidate_pairs(x: np.ndarray, nm: int, radius: float) -> np.ndarray:
    xw = np.mod(x.astype(np.float64), nm)
    xw[xw >= nm] = 0.0
    tree = cKDTree(xw.T, boxsize=nm)
    return tree.query_pairs(radius, output_type="ndarray")


def labels_from_pairs(n: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    g = coo_matrix((np.ones(len(a)), (a, b)), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    lab = np.full(comp.max() + 1, n, dtype=np.int64)
    np.minimum.at(lab, comp, np.arange(n))
    return lab[comp].astype(np.int32)


def fof_labels(disp: np.ndarray, np_side: int, nm: int, b_frac: float = 0.2) -> np.ndarray:
    """Group label (smallest id in the group) of every particle."""
    x = positions_fp32(disp, np_side, nm)
    b2 = link_length_sq(b_frac, np_side, nm)
    pairs = candidate_pairs(x, nm, float(np.sqrt(np.float64(b2))) * (1 + 1e-5) + 1e-6)
    if len(pairs):
        keep = r2_fp32(x, pairs[:, 0], pairs[:, 1], nm) <= b2
        pairs = pairs[keep]
    n = np_side ** 3
    if not len(pairs):
        return np.arange(n, dtype=np.int32)
    return labels_from_pairs(n, pairs[:, 0], pairs[:, 1])


def fof_labels_brute(disp: np.ndarray, np_side: int, nm: int, b_frac: float = 0.2) -> np.ndarray:
    """All pairs, for tiny inputs: the same float32 test, no tree."""
    x = positions_fp32(disp, np_side, nm)
    b2 = link_length_sq(b_frac, np_side, nm)
    n = x.shape[1]
    a, b = np.triu_indices(n, 1)
    keep = r2_fp32(x, a, b, nm) <= b2
    return labels_from_pairs(n, a[keep], b[keep])


def halo_catalogue(disp: np.ndarray, vel, labels: np.ndarray, np_side: int, nm: int, min_members: int):
    """Groups with at least ``min_members`` particles, in increasing root id:
    root id, member count, centre of mass (mesh units, in [0, nm)) and mean
    velocity.  The centre is the root's position plus the mean nearest-image
    offset of the members from the root (groups may straddle the box edge);
    float64 from the float32 positions."""
    x = positions_fp32(disp, np_side, nm).astype(np.float64)
    counts = np.bincount(labels, minlength=labels.size)
    roots = np.flatnonzero(counts >= min_members)
    com = np.zeros((3, len(roots)))
    vmean = np.zeros((3, len(roots)))
    order = np.argsort(labels, kind="stable")
    starts = np.searchsorted(labels[order], roots)
    for h, (r, s) in enumerate(zip(roots, starts)):
        m = order[s:s + counts[r]]
        rel = x[:, m] - x[:, [r]]
        rel -= nm * np.rint(rel / nm)
        com[:, h] = np.mod(x[:, r] + rel.mean(axis=1), nm)
        if vel is not None:
            vmean[:, h] = vel[:, m].astype(np.float64).mean(axis=1)
    return roots.astype(np.int32), counts[roots].astype(np.int32), com, vmean
