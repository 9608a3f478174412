"""Replays of a captured step graph against the same steps taken eagerly.

Each replay is followed by unrelated eager device work and a synchronisation,
and every replay is compared with the eager state after the same number of
steps: bit for bit with the deterministic (segmented) assembly, to round-off
with the atomic one."""
import numpy as np
import pytest
import torch

import otm_workloads as W
from tests.gpu_common import make_sim, require_gpu
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu

FIELDS = ("x", "du", "m", "f", "xp", "vol", "sigma", "epsbar", "T", "N", "dN", "lam")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _pair(w, scatter):
    eager, _ = make_sim(w, scatter=scatter)
    graphed, _ = make_sim(w, scatter=scatter)
    for s in (eager, graphed):
        s.init()
        s.step()                      # loads every kernel before the capture
    return eager, graphed


@pytest.mark.parametrize("scatter", ["segmented", "atomic"])
def test_step_graph_replays_match_eager_steps(scatter):
    w = W.config_by_name("small_rod")
    eager, graphed = _pair(w, scatter)
    g = graphed.capture(steps=3)
    for r in range(4):
        g.replay()
        noise = torch.randn(4096, device="cuda")
        float((noise * noise).sum())          # eager work and a sync between replays
        eager.run(3)
        a, b = eager.fields(), graphed.fields()
        assert graphed.n == eager.n == 1 + 3 * (r + 1)
        for k in FIELDS:
            if scatter == "segmented":
                assert np.array_equal(a[k], b[k]), (r, k)
            else:
                # positions as displacements (absolute positions would hide errors)
                x0 = {"x": w.x_nodes, "xp": w.x_mp}.get(k, 0.0)
                err = rel_err(b[k] - x0, a[k] - x0)
                assert err < 1e-11, (r, k, err)
    eager.check_diag()
    graphed.check_diag()


def test_cutting_step_graph_replays_match_eager_steps():
    """The chip-formation step (tool contact, its device clock, fracture) in a
    captured graph: 5 replays of 6 steps of the small cut against eager steps,
    bit for bit with the segmented assembly, failure flags, tangential gaps
    and clock included."""
    w = W.config_by_name("small_cut")
    eager, graphed = _pair(w, "segmented")
    g = graphed.capture(steps=6)
    for r in range(5):
        g.replay()
        eager.run(6)
        a, b = eager.fields(), graphed.fields()
        for k in FIELDS + ("failed", "gT"):
            assert np.array_equal(a[k], b[k]), (r, k)
        assert a["clock"] == b["clock"]
    assert b["failed"].sum() > 0 or (np.abs(b["gT"]).sum() > 0)
    eager.check_diag()
    graphed.check_diag()


def test_graph_replay_after_erosion_raises():
    """Erosion shrinks the MP arrays and their component stride: a graph
    captured before it must not replay."""
    w = W.config_by_name("small_cut")
    sim, _ = make_sim(w)
    sim.init()
    sim.step()
    g = sim.capture(steps=1)
    g.replay()
    sim.erode()
    with pytest.raises(RuntimeError, match="capture the steps again"):
        g.replay()
    g2 = sim.capture(steps=1)
    g2.replay()
    sim.check_diag()
