"""Float32 replay of the deterministic CIC mass deposit (Sec. 3.3 CIC).

Test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use this module.

The FP64 oracle (``pm.cic_deposit``) fixes *what* the deposit computes.  This
module fixes, in addition, every float32 rounding, so that a float32
implementation that follows the same rule can be checked bit for bit.  The
rule is a reading (the paper states no summation order); it is chosen so
that the result does not depend on any order at all:

Positions are stored as float32 displacements d (in mesh cells) from the
Lagrangian lattice; particle id p = (i*N + j)*N + k, lattice point of axis e
at i_e * Nm / Np cells.  Mesh nodes sit at cell centres, so the node
coordinate of a particle is u = i_e Nm / Np - 1/2 + d_e.  Per axis e:
    qi  = (i_e * Nm) div Np                         (integer)
    rem = (i_e * Nm) mod Np
    qf  = float32(2 rem - Np) / float32(2 Np)       (one float32 divide; -1/2
                                                     exactly when Nm/Np is whole)
    u   = qf + d_e                                  (float32 add)
    fl  = floor(u);  f = u - fl                     (float32)
    c_e = (qi + fl) mod Nm                          (home cell)
    w_0 = 1 - f,  w_1 = f                           (float32)
For the 8 offsets s = (sx, sy, sz), k = 4 sx + 2 sy + sz:
    w_s = (w_sx(fx) * w_sy(fy)) * w_sz(fz)          (float32, no fused multiply-add)
    q_s = rint(w_s * 2^32)                          (unsigned 64-bit; ties to even)
Node n = c + s holds the integer sum S(n) of the q_s of every particle and
offset that reach it (exact, so independent of the order of the terms), and
    rho(n)   = float32(S(n)) * 2^-32                (one rounding to nearest even)
    delta(n) = rho(n) * c_inv - 1.0f,  c_inv = float32(Nm^3 / Np)
(two float32 roundings, no fused multiply-add).  A weight w >= 2^-9 is a
multiple of 2^-32, so q_s is exact and rho(n) is the correctly rounded exact
sum of the node's float32 weights; smaller weights are rounded to 2^-32.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32
FIX_SCALE = 2.0 ** 32


def _axis_terms(np_side: int, nm: int):
    i = np.arange(np_side, dtype=np.int64)
    qi = (i * nm) // np_side
    rem = (i * nm) % np_side
    qf = (2 * rem - np_side).astype(F32) / F32(2 * np_side)
    return qi, qf


def home_cells(disp: np.ndarray, np_side: int, nm: int, pid=None):
    """disp: (3, n) float32 in mesh cells of particles pid (default: all,
    n = Np^3).  Returns cells (3, n) int64, f (3, n) f32."""
    disp = np.asarray(disp, dtype=F32)
    qi, qf = _axis_terms(np_side, nm)
    if pid is None:
        pid = np.arange(np_side ** 3, dtype=np.int64)
    lat = [pid // (np_side * np_side), (pid // np_side) % np_side, pid % np_side]
    cells, fr = [], []
    for e in range(3):
        u = qf[lat[e]] + disp[e]
        fl = np.floor(u)
        fr.append(u - fl)
        cells.append(np.mod(qi[lat[e]] + fl.astype(np.int64), nm))
    return np.stack(cells), np.stack(fr)


def weights(f: np.ndarray):
    """(8, n) float32 weights in offset order k = 4 sx + 2 sy + sz."""
    one = F32(1.0)
    w = [[one - f[e], f[e]] for e in range(3)]
    out = np.empty((8, f.shape[1]), dtype=F32)
    for k in range(8):
        sx, sy, sz = (k >> 2) & 1, (k >> 1) & 1, k & 1
        xy = (w[0][sx] * w[1][sy]).astype(F32)
        out[k] = (xy * w[2][sz]).astype(F32)
    return out


def fixed_point(w: np.ndarray) -> np.ndarray:
    """q = rint(w * 2^32) as uint64 (w float32 in [0, 1]; the product is exact)."""
    return np.rint(w.astype(np.float64) * FIX_SCALE).astype(np.uint64)


def _node_index(cells: np.ndarray, k: int, nm: int) -> np.ndarray:
    s = ((k >> 2) & 1, (k >> 1) & 1, k & 1)
    return (((cells[0] + s[0]) % nm) * nm + (cells[1] + s[1]) % nm) * nm + (cells[2] + s[2]) % nm


def _to_rho(S: np.ndarray) -> np.ndarray:
    """float32(S) * 2^-32 with one rounding of S (exact through float64 below 2^53)."""
    assert S.size == 0 or int(S.max()) < (1 << 53)
    return (S.astype(np.float64).astype(F32) * F32(2.0 ** -32)).astype(F32)


def _contrast(rho: np.ndarray, np_side: int, nm: int) -> np.ndarray:
    c_inv = F32(nm ** 3 / np_side ** 3)
    return ((rho * c_inv).astype(F32) - F32(1.0)).astype(F32)


def node_sums(disp, np_side: int, nm: int, pid=None) -> np.ndarray:
    """S(n) for every node (nm^3 uint64, flat C order) of the particles pid."""
    cells, f = home_cells(disp, np_side, nm, pid)
    q = fixed_point(weights(f))
    S = np.zeros(nm ** 3, dtype=np.uint64)
    for k in range(8):
        np.add.at(S, _node_index(cells, k, nm), q[k])
    return S


def density(disp, np_side: int, nm: int, contrast=True) -> np.ndarray:
    """rho (or delta) on the nm^3 mesh, float32."""
    rho = _to_rho(node_sums(disp, np_side, nm)).reshape(nm, nm, nm)
    return _contrast(rho, np_side, nm) if contrast else rho


def density_at_nodes_chunked(disp, np_side: int, nm: int, nodes, contrast=True, chunk=1 << 26,
                             progress=None):
    """The same result at the given nodes ((M, 3) int) only, scanning the
    particles ``chunk`` at a time (for counts whose temporaries do not fit in
    host memory at once).  ``progress(done, total)`` is called after every
    chunk when given."""
    nodes = np.asarray(nodes, dtype=np.int64).reshape(-1, 3)
    want = (nodes[:, 0] * nm + nodes[:, 1]) * nm + nodes[:, 2]
    uniq, inv = np.unique(want, return_inverse=True)
    S = np.zeros(len(uniq), dtype=np.uint64)
    n_all = disp.shape[1]
    for a in range(0, n_all, chunk):
        b = min(n_all, a + chunk)
        pid = np.arange(a, b, dtype=np.int64)
        cells, f = home_cells(disp[:, a:b], np_side, nm, pid)
        q = fixed_point(weights(f))
        for k in range(8):
            idx = _node_index(cells, k, nm)
            pos = np.minimum(np.searchsorted(uniq, idx), len(uniq) - 1)
            m = uniq[pos] == idx
            np.add.at(S, pos[m], q[k][m])
        if progress is not None:
            progress(b, n_all)
    rho = _to_rho(S)[inv]
    return _contrast(rho, np_side, nm) if contrast else rho


def density_at_nodes(disp, np_side: int, nm: int, nodes: np.ndarray, contrast=True):
    """``density`` at the given nodes only ((M, 3) int)."""
    return density_at_nodes_chunked(disp, np_side, nm, nodes, contrast, chunk=1 << 62)
