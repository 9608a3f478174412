"""Pins of the oracle's support-domain search (Alg. 3) against its definition."""
import json
import os

import numpy as np
import pytest

from oracle import search
import otm_workloads as inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "search_tiny.json")


def _rows(offsets, idx):
    return [list(idx[offsets[i]:offsets[i + 1]]) for i in range(len(offsets) - 1)]


def test_golden_tiny_inclusive_boundary():
    g = json.load(open(GOLDEN))
    X = np.array(g["nodes"], float)
    P = np.array(g["mps"], float)
    r = g["radius"]
    for fn in (lambda: search.neighbors_bruteforce(X, P, r),
               lambda: search.neighbors_linked_cell(X, P, r, r)):
        off, idx = fn()
        assert _rows(off, idx) == g["expected"]
    for k, p in enumerate(P):
        assert list(search.neighbors_one(X, p, r)) == g["expected"][k]


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_linked_cell_equals_bruteforce_random(seed):
    X, P = inputs.random_cloud(400, 300, seed)
    # some MPs outside the node box exercise the clamped edge cells
    P[:20] = P[:20] * 1.4 - 0.2
    for r, cs in ((0.11, 0.11), (0.2, 0.25), (0.05, 0.3)):
        o1, i1 = search.neighbors_bruteforce(X, P, r)
        o2, i2 = search.neighbors_linked_cell(X, P, r, cs)
        assert np.array_equal(o1, o2) and np.array_equal(i1, i2)
        assert i1.dtype == np.int32 and o1.dtype == np.int64


def test_linked_cell_equals_bruteforce_cube(cube):
    r = cube.r_list
    o1, i1 = search.neighbors_bruteforce(cube.x_nodes, cube.x_mp, r)
    o2, i2 = search.neighbors_linked_cell(cube.x_nodes, cube.x_mp, r, r * 1.0001)
    assert np.array_equal(o1, o2) and np.array_equal(i1, i2)
    K = np.diff(o1)
    # every tet-centroid MP sees at least the 4 corners of its tet
    assert K.min() >= 4
    # rows are strictly ascending (canonical order, no duplicates)
    for a, b in zip(o1[:-1], o1[1:]):
        assert np.all(np.diff(i1[a:b]) > 0)


def test_search_rejects_small_cells():
    X, P = inputs.random_cloud(10, 10, 0)
    with pytest.raises(ValueError):
        search.neighbors_linked_cell(X, P, 0.3, 0.2)


def test_influence_lists_transpose(cube):
    off, idx = search.neighbors_bruteforce(cube.x_nodes, cube.x_mp, cube.r_list)
    starts, pairs = search.influence_lists(cube.n_nodes, off, idx)
    mp_of_pair = np.repeat(np.arange(cube.n_mp), np.diff(off))
    for I in (0, 17, 555, 999):
        q = pairs[starts[I]:starts[I + 1]]
        assert np.all(idx[q] == I)
        assert np.all(np.diff(q) > 0)
        # brute force: MPs whose support contains I
        expect = [p for p in range(cube.n_mp) if I in idx[off[p]:off[p + 1]]]
        assert list(mp_of_pair[q]) == expect
