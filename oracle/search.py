"""Support-domain search (Sec. 3, linked-cell method, Alg. 3).

The support domain of a material point p is the set of nodes I with
|x_p - x_I| <= r (inclusive).  The squared distance is evaluated as
((dx*dx + dy*dy) + dz*dz) with dx = x_p - x_I, every operation rounded on its
own (NumPy never fuses a multiply into an add), so that the set is a function
of the float64 inputs alone.  Lists are returned in canonical order: CSR over
material points, node indices ascending within each row.
"""
from __future__ import annotations

import numpy as np


def _sqdist(xp, xn):
    dx = xp[..., 0] - xn[..., 0]
    dy = xp[..., 1] - xn[..., 1]
    dz = xp[..., 2] - xn[..., 2]
    return (dx * dx + dy * dy) + dz * dz


def _csr_from_pairs(n_mp, mp_of_pair, node_of_pair):
    order = np.lexsort((node_of_pair, mp_of_pair))
    mp_sorted = mp_of_pair[order]
    idx = node_of_pair[order].astype(np.int32)
    counts = np.bincount(mp_sorted, minlength=n_mp)
    offsets = np.zeros(n_mp + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    return offsets, idx


def neighbors_bruteforce(x_nodes, x_mp, r):
    """Definition of the support domain: test every (MP, node) pair."""
    x_nodes = np.asarray(x_nodes, np.float64)
    x_mp = np.asarray(x_mp, np.float64)
    r2 = r * r
    mps, nodes = [], []
    chunk = max(1, 4_000_000 // max(1, x_nodes.shape[0]))
    for s in range(0, x_mp.shape[0], chunk):
        d2 = _sqdist(x_mp[s:s + chunk, None, :], x_nodes[None, :, :])
        p, i = np.nonzero(d2 <= r2)
        mps.append(p + s)
        nodes.append(i)
    mp_of_pair = np.concatenate(mps) if mps else np.zeros(0, np.int64)
    node_of_pair = np.concatenate(nodes) if nodes else np.zeros(0, np.int64)
    return _csr_from_pairs(x_mp.shape[0], mp_of_pair, node_of_pair)


def neighbors_one(x_nodes, xp, r):
    """Support domain of a single material point (ascending node ids)."""
    d2 = _sqdist(np.asarray(xp, np.float64)[None, :], np.asarray(x_nodes, np.float64))
    return np.nonzero(d2 <= r * r)[0].astype(np.int32)


def cell_grid(x_nodes, cell_size):
    """Static cells over the node bounding box (Alg. 3, step 1)."""
    lo = x_nodes.min(axis=0)
    hi = x_nodes.max(axis=0)
    dims = np.floor((hi - lo) / cell_size).astype(np.int64) + 1
    return lo, dims


def cell_coords(x, lo, cell_size, dims):
    c = np.floor((x - lo) / cell_size).astype(np.int64)
    return np.clip(c, 0, dims - 1)


def neighbors_linked_cell(x_nodes, x_mp, r, cell_size):
    """Linked-cell search (Alg. 3): bin nodes into cells of edge
    ``cell_size >= r``, then test only the nodes of the 27 cells around the
    cell of each material point.  Returns the same canonical CSR as the
    brute-force definition."""
    if cell_size < r:
        raise ValueError("cell edge must be at least the search radius")
    x_nodes = np.asarray(x_nodes, np.float64)
    x_mp = np.asarray(x_mp, np.float64)
    n_mp = x_mp.shape[0]
    if n_mp == 0:                       # no material points: no supports
        return np.zeros(1, np.int64), np.zeros(0, np.int32)
    lo, dims = cell_grid(x_nodes, cell_size)
    cn = cell_coords(x_nodes, lo, cell_size, dims)
    cid = (cn[:, 2] * dims[1] + cn[:, 1]) * dims[0] + cn[:, 0]
    order = np.argsort(cid, kind="stable")
    n_cells = int(np.prod(dims))
    cell_start = np.zeros(n_cells + 1, dtype=np.int64)
    np.cumsum(np.bincount(cid, minlength=n_cells), out=cell_start[1:])
    max_per_cell = int(np.diff(cell_start).max())

    cp = cell_coords(x_mp, lo, cell_size, dims)
    r2 = r * r
    mps, nodes = [], []
    for oz in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                c = cp + np.array([ox, oy, oz])
                ok = np.all((c >= 0) & (c < dims), axis=1)
                pids = np.nonzero(ok)[0]
                cc = c[ok]
                ci = (cc[:, 2] * dims[1] + cc[:, 1]) * dims[0] + cc[:, 0]
                s0, s1 = cell_start[ci], cell_start[ci + 1]
                for k in range(max_per_cell):
                    has = s0 + k < s1
                    if not has.any():
                        break
                    p = pids[has]
                    nd = order[s0[has] + k]
                    hit = _sqdist(x_mp[p], x_nodes[nd]) <= r2
                    mps.append(p[hit])
                    nodes.append(nd[hit])
    mp_of_pair = np.concatenate(mps)
    node_of_pair = np.concatenate(nodes)
    return _csr_from_pairs(n_mp, mp_of_pair, node_of_pair)


def influence_lists(n_nodes, offsets, idx):
    """Influence domain of every node (Sec. 2.1): the transpose of the
    support lists, entries = pair ids in ascending order."""
    order = np.argsort(idx, kind="stable")
    counts = np.bincount(idx, minlength=n_nodes)
    starts = np.zeros(n_nodes + 1, dtype=np.int64)
    np.cumsum(counts, out=starts[1:])
    return starts, order.astype(np.int64)
