"""Pins of the oracle's node management at erosion (Sec. 3.3 adds and
deletes nodes; the cutting workload adds nodes at the freed surfaces):
insertion where material was removed and deletion of nodes that no support
holds any more.

* Every inserted node sits at a removed MP, farther than delta from every
  node that existed before (brute force over all nodes, not the support
  lists the rule reads), and every removed MP that left no node has an old
  node or a removed MP of smaller index within delta.
* The inserted node's increment is the interpolated increment: exact for a
  linear increment field (LME linear reproduction).
* Lumped mass stays conserved (partition of unity), node positions and
  increments of the old nodes are untouched.
* Deletion: on a body cut in two, the nodes farther than the search radius
  from every remaining MP (brute force) are exactly the deleted ones, the
  renumbered lists equal a fresh search over the remaining nodes, and the
  next step's MP fields equal those of the same run without deletion.
"""
import numpy as np
import pytest

import otm_workloads as W
from oracle import search, step as OST


def _d2(a, b):
    return search._sqdist(a[:, None, :], b[None, :, :])


@pytest.fixture(scope="module")
def cut_at_45():
    w = W.config_by_name("small_cut")
    p = W.params_from_workload(w, insert_dist=0.5 * w.h, delete_orphans=True)
    st = OST.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    for _ in range(45):
        OST.step(st, p)
    assert st.failed.sum() > 10
    return w, p, st


def test_inserted_nodes_follow_the_rule_by_brute_force(cut_at_45):
    w, p, st0 = cut_at_45
    st = st0.copy()
    delta2 = p["insert_dist"] ** 2
    removed = np.nonzero(st.failed)[0]
    x_old, du_old = st.x.copy(), st.du.copy()
    m_total = st.mass[~st.failed].sum()
    OST.erode(st, p)
    ins, dele = st.node_events
    n0 = x_old.shape[0]
    assert ins > 0 and dele == 0
    assert st.x.shape[0] == n0 + ins
    new = st.x[n0:]
    # each new node sits at a removed MP, far from every old node
    src = [int(np.nonzero((st0.xp[removed] == xn).all(axis=1))[0][0]) for xn in new]
    assert len(set(src)) == ins and src == sorted(src)
    assert (_d2(new, x_old).min(axis=1) > delta2).all()
    # every removed MP without a node: an old node or an earlier removed MP near it
    placed = set(src)
    xr = st0.xp[removed]
    for k in range(removed.size):
        if k in placed:
            continue
        near_old = _d2(xr[k:k + 1], x_old).min() <= delta2
        near_earlier = k > 0 and _d2(xr[k:k + 1], xr[:k]).min() <= delta2
        assert near_old or near_earlier, k
    # old nodes untouched, mass conserved
    assert np.array_equal(st.x[:n0], x_old) and np.array_equal(st.du[:n0], du_old)
    assert abs(st.m.sum() - m_total) <= 1e-12 * m_total
    assert (st.m[n0:] > 0).all()


def test_inserted_increment_reproduces_a_linear_field(cut_at_45):
    w, p, st0 = cut_at_45
    st = st0.copy()
    A = np.array([[1e-3, 2e-4, 0.0], [-5e-4, 3e-4, 1e-4], [2e-4, 0.0, -1e-3]])
    b = np.array([1e-9, -2e-9, 5e-10])
    st.du = st.x @ A.T + b
    n0 = st.x.shape[0]
    OST.erode(st, p)
    new = st.x[n0:]
    assert new.shape[0] > 0
    want = new @ A.T + b
    assert np.abs(st.du[n0:] - want).max() <= 1e-12 * np.abs(want).max()


def test_orphan_nodes_are_deleted_and_lists_renumbered():
    """The small cut's workpiece with every MP above a horizontal cut
    failed: the nodes that only those MPs held are orphans."""
    w = W.config_by_name("small_cut")
    p = W.params_from_workload(w, delete_orphans=True)
    pk = W.params_from_workload(w)
    st = OST.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    for _ in range(3):
        OST.step(st, p)
    y_cut = np.quantile(st.xp[:, 1], 0.6)
    st.failed = st.xp[:, 1] > y_cut
    keep_run = st.copy()
    x_before = st.x.copy()
    OST.erode(st, p)
    OST.erode(keep_run, pk)
    _, dele = st.node_events
    assert dele > 0 and keep_run.node_events == (0, 0)
    # the deleted nodes are exactly those out of reach of every remaining MP
    reach = _d2(x_before, st.xp).min(axis=1) <= p["r_list"] ** 2
    assert dele == int((~reach).sum())
    assert np.array_equal(st.x, x_before[reach])
    # renumbered lists = a fresh search over the remaining nodes
    off, idx = search.neighbors_bruteforce(st.x, st.xp, p["r_list"])
    assert np.array_equal(off, st.offsets) and np.array_equal(idx, st.idx)
    assert (st.m > 0).all()
    # the next step does not see the orphans: MP fields as without deletion
    OST.step(st, p)
    OST.step(keep_run, pk)
    for k in ("xp", "vol", "F", "be", "sigma", "epsbar", "T", "N", "dN", "lam"):
        assert np.array_equal(getattr(st, k), getattr(keep_run, k)), k
    assert np.array_equal(st.x, keep_run.x[reach])
