"""Node management at erosion on the GPU against the oracle: nodes added at
the freed surface (insert_dist) over two erosions of the small cut (five
steps after the last), and the nodes in no support deleted (delete_orphans) after a whole part is cut off;
both assemblies, float64 within 1e-10, with identical lists, node counts and
failure flags."""
import json

import numpy as np
import pytest
import torch

import otm_workloads as W
from oracle import step as OST
from tests.gpu_common import make_sim, require_gpu
from tests.helpers import compare, gpu_fields, oracle_fields

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
ERODE_AT = (30, 45)
STEPS = 50


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _over(w):
    return dict(insert_dist=0.5 * w.h)


@pytest.fixture(scope="module")
def oracle_run():
    """The oracle's run, and the reference position of every node (an added
    node's position when it was added), for displacements."""
    w = W.config_by_name("small_cut")
    p = W.params_from_workload(w, **_over(w))
    st = OST.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    orig = np.arange(w.n_mp)
    events = []
    x0 = w.x_nodes.copy()
    for s in range(1, STEPS + 1):
        OST.step(st, p)
        if s in ERODE_AT:
            orig = orig[~st.failed]
            n_before = st.x.shape[0]
            OST.erode(st, p)
            events.append(st.node_events)
            x0 = np.concatenate([x0, st.x[n_before:]])
    assert sum(e[0] for e in events) > 0
    return w, p, st, orig, events, x0


@pytest.mark.parametrize("scatter", ["atomic", "segmented"])
def test_node_insertion_matches_oracle(oracle_run, scatter):
    w, p, st, orig, events, x0 = oracle_run
    print(f"node insertion, {scatter}: erosions at {ERODE_AT}, oracle events {events}",
          flush=True)
    sim, _ = make_sim(w, scatter=scatter, **_over(w))
    sim.init()
    got = []
    for s in range(1, STEPS + 1):
        sim.step()
        if s in ERODE_AT:
            sim.erode()
            got.append(sim.node_events)
    sim.check_diag()
    assert got == events
    g = sim.fields()
    assert sim.n_nodes == st.x.shape[0] and sim.n_mp == st.xp.shape[0]
    assert np.array_equal(g["offsets"], st.offsets) and np.array_equal(g["idx"], st.idx)
    assert np.array_equal(g["failed"], st.failed)
    errs = compare(gpu_fields(g, x0, w.x_mp[orig], p["T_r"]),
                   oracle_fields(st, x0, w.x_mp[orig], p["T_r"]))
    print(json.dumps({k: float(v) for k, v in errs.items()}))
    bad = {k: v for k, v in errs.items() if not v < FP64_TOL}
    assert not bad, bad


@pytest.mark.parametrize("scatter", ["atomic", "segmented"])
def test_orphan_deletion_matches_oracle(scatter):
    """After 30 steps every MP above a horizontal cut is marked failed: the
    nodes only they held are deleted and the lists renumbered; two steps later
    GPU and oracle agree."""
    w = W.config_by_name("small_cut")
    p = W.params_from_workload(w, delete_orphans=True)
    st = OST.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    for _ in range(30):
        OST.step(st, p)
    y_cut = np.quantile(st.xp[:, 1], 0.6)
    cut = st.failed | (st.xp[:, 1] > y_cut)
    failed_before = st.failed.copy()
    st.failed = cut.copy()
    orig = np.nonzero(~cut)[0]
    OST.erode(st, p)
    assert st.node_events[1] > 0
    for _ in range(2):
        OST.step(st, p)
    print(f"orphan deletion, {scatter}: {st.node_events[1]} nodes", flush=True)
    sim, _ = make_sim(w, scatter=scatter, delete_orphans=True)
    sim.init()
    for _ in range(30):
        sim.step()
    assert np.array_equal(sim.failed.cpu().numpy().astype(bool), failed_before)
    sim.failed.copy_(torch.from_numpy(cut.astype(np.int32)))
    sim.erode()
    assert sim.node_events == st.node_events
    sim.run(2)
    sim.check_diag()
    g = sim.fields()
    assert sim.n_nodes == st.x.shape[0]
    assert np.array_equal(g["offsets"], st.offsets) and np.array_equal(g["idx"], st.idx)
    errs = compare(gpu_fields(g, st.x * 0, w.x_mp[orig], p["T_r"]),
                   oracle_fields(st, st.x * 0, w.x_mp[orig], p["T_r"]))
    bad = {k: v for k, v in errs.items() if not v < FP64_TOL}
    assert not bad, bad
