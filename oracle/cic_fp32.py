"""Float32 same-order replay of the deterministic CIC deposit (Sec. 3.3 CIC).

The FP64 oracle (``pm.cic_deposit``) fixes *what* the deposit computes.  This
module fixes, in addition, the exact float32 rounding sequence, so that a
float32 implementation that follows the same order can be checked bit for
bit.  The order is a reading (the paper does not state one):

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
For the 8 offsets s = (sx, sy, sz), taken in the order k = 4 sx + 2 sy + sz:
    w_s = (w_sx(fx) * w_sy(fy)) * w_sz(fz)          (float32, no fused multiply-add)
Per home cell c and offset s, the partial sum P_s(c) adds w_s of the cell's
particles in ascending particle id, starting from 0.0f.
Node n then adds its 8 source cells in ascending cell order, i.e.
rho(n) = 0.0f + P_s7(n - s7) + P_s6(n - s6) + ... + P_s0(n - s0), offsets
k = 7 .. 0 (a cell without particles contributes +0.0f).
The density contrast is delta = rho * c_inv - 1.0f, c_inv = float32(Nm^3 / Np)
(two float32 roundings, no fused multiply-add).
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


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
    """(8, Np) float32 weights in offset order k = 4 sx + 2 sy + sz."""
    one = F32(1.0)
    w = [[one - f[e], f[e]] for e in range(3)]
    out = np.empty((8, f.shape[1]), dtype=F32)
    for k in range(8):
        sx, sy, sz = (k >> 2) & 1, (k >> 1) & 1, k & 1
        xy = (w[0][sx] * w[1][sy]).astype(F32)
        out[k] = (xy * w[2][sz]).astype(F32)
    return out


def cell_partials(disp, np_side: int, nm: int):
    """P_s(c) for all cells: (8, nm, nm, nm) float32, sums in ascending id."""
    cells, f = home_cells(disp, np_side, nm)
    w = weights(f)
    flat = (cells[0] * nm + cells[1]) * nm + cells[2]
    order = np.argsort(flat, kind="stable")          # ascending id within a cell
    fs = flat[order]
    first = np.r_[0, np.flatnonzero(np.diff(fs)) + 1]
    rank = np.arange(len(fs)) - np.repeat(first, np.diff(np.r_[first, len(fs)]))
    P = np.zeros((8, nm ** 3), dtype=F32)
    for r in range(int(rank.max()) + 1 if len(rank) else 0):
        sel = order[rank == r]
        cidx = flat[sel]                              # unique at a given rank
        for k in range(8):
            P[k, cidx] = P[k, cidx] + w[k, sel]
    return P.reshape(8, nm, nm, nm)


def density(disp, np_side: int, nm: int, contrast=True) -> np.ndarray:
    """rho (or delta) on the nm^3 mesh, float32, in the documented order."""
    P = cell_partials(disp, np_side, nm)
    rho = np.zeros((nm, nm, nm), dtype=F32)
    for k in range(7, -1, -1):
        s = ((k >> 2) & 1, (k >> 1) & 1, k & 1)
        rho = rho + np.roll(P[k], shift=s, axis=(0, 1, 2))
    if not contrast:
        return rho
    c_inv = F32(nm ** 3 / np_side ** 3)
    return (rho * c_inv).astype(F32) - F32(1.0)


def density_at_nodes(disp, np_side: int, nm: int, nodes: np.ndarray, contrast=True):
    """Same result as ``density`` but only at the given nodes ((M, 3) int)."""
    cells, f = home_cells(disp, np_side, nm)
    w = weights(f)
    flat = (cells[0] * nm + cells[1]) * nm + cells[2]
    order = np.argsort(flat, kind="stable")
    fs = flat[order]
    out = np.empty(len(nodes), dtype=F32)
    for j, n in enumerate(np.asarray(nodes)):
        rho = F32(0.0)
        for k in range(7, -1, -1):
            s = np.array([(k >> 2) & 1, (k >> 1) & 1, k & 1])
            c = np.mod(n - s, nm)
            cf = (c[0] * nm + c[1]) * nm + c[2]
            lo, hi = np.searchsorted(fs, cf, "left"), np.searchsorted(fs, cf, "right")
            part = F32(0.0)
            for p in order[lo:hi]:
                part = F32(part + w[k, p])
            rho = F32(rho + part)
        out[j] = rho
    if contrast:
        c_inv = F32(nm ** 3 / np_side ** 3)
        out = (out * c_inv).astype(F32) - F32(1.0)
    return out


def density_at_nodes_chunked(disp, np_side: int, nm: int, nodes, contrast=True, chunk=1 << 26,
                             progress=None):
    """``density_at_nodes`` for particle counts too large to hold every
    temporary at once: particles are scanned in id order, ``chunk`` at a
    time, keeping only those whose home cell feeds one of the nodes; the
    kept ones (still in ascending id) then go through the same replay.
    ``progress(done, total)`` is called after every chunk when given."""
    nodes = np.asarray(nodes, dtype=np.int64)
    feed = set()
    for n in nodes:
        for k in range(8):
            s = np.array([(k >> 2) & 1, (k >> 1) & 1, k & 1])
            c = np.mod(n - s, nm)
            feed.add(int((c[0] * nm + c[1]) * nm + c[2]))
    feed = np.array(sorted(feed), dtype=np.int64)
    n_all = disp.shape[1]
    keep_id, keep_cells, keep_f = [], [], []
    for a in range(0, n_all, chunk):
        b = min(n_all, a + chunk)
        pid = np.arange(a, b, dtype=np.int64)
        cells, f = home_cells(disp[:, a:b], np_side, nm, pid)
        flat = (cells[0] * nm + cells[1]) * nm + cells[2]
        pos = np.minimum(np.searchsorted(feed, flat), len(feed) - 1)
        m = feed[pos] == flat
        keep_id.append(pid[m])
        keep_cells.append(cells[:, m])
        keep_f.append(f[:, m])
        if progress is not None:
            progress(b, n_all)
    cells = np.concatenate(keep_cells, axis=1)
    f = np.concatenate(keep_f, axis=1)
    w = weights(f)
    flat = (cells[0] * nm + cells[1]) * nm + cells[2]
    order = np.argsort(flat, kind="stable")      # ids ascend within a cell
    fs = flat[order]
    out = np.empty(len(nodes), dtype=F32)
    for j, n in enumerate(nodes):
        rho = F32(0.0)
        for k in range(7, -1, -1):
            s = np.array([(k >> 2) & 1, (k >> 1) & 1, k & 1])
            c = np.mod(n - s, nm)
            cf = (c[0] * nm + c[1]) * nm + c[2]
            lo, hi = np.searchsorted(fs, cf, "left"), np.searchsorted(fs, cf, "right")
            part = F32(0.0)
            for q in order[lo:hi]:
                part = F32(part + w[k, q])
            rho = F32(rho + part)
        out[j] = rho
    if contrast:
        c_inv = F32(nm ** 3 / np_side ** 3)
        out = (out * c_inv).astype(F32) - F32(1.0)
    return out

