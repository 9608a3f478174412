"""Chip formation (Sec. 4.2) on the GPU against the oracle: the small cut
(40 x 24 um piece, tool moving in at 50 m/s, low fracture strain) for 60
float64 steps with both assemblies, so that tool contact with stick and slip,
plastic flow and fracture all happen; and the full-size slab for a few steps."""
import json

import numpy as np
import pytest

import otm_workloads as W
from oracle import contact as OC
from oracle import step as OST
from tests.gpu_common import make_sim, require_gpu
from tests.helpers import compare, gpu_fields, oracle_fields, rel_err

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def small_cut():
    w = W.config_by_name("small_cut")
    p = W.params_from_workload(w)
    st = OST.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    for _ in range(w.steps):
        OST.step(st, p)
    g, _ = OC.tool_gap(st.x, st.clock, p)
    assert st.failed.sum() > 10 and (g < 0).sum() > 5
    return w, p, st


@pytest.mark.parametrize("scatter", ["atomic", "segmented"])
def test_small_cut_60_steps_fp64(small_cut, scatter):
    w, p, st = small_cut
    sim, _ = make_sim(w, scatter=scatter)
    sim.init()
    sim.run(w.steps)
    sim.check_diag()
    g = sim.fields()
    assert np.array_equal(g["offsets"], st.offsets) and np.array_equal(g["idx"], st.idx)
    assert np.array_equal(g["failed"], st.failed)
    errs = compare(gpu_fields(g, w.x_nodes, w.x_mp, p["T_r"]),
                   oracle_fields(st, w.x_nodes, w.x_mp, p["T_r"]))
    errs["gT"] = rel_err(g["gT"], st.gT)
    print("small cut, 60 steps:", json.dumps({k: float(v) for k, v in errs.items()}),
          "failed", int(st.failed.sum()))
    bad = {k: v for k, v in errs.items() if not v < FP64_TOL}
    assert not bad, bad
    assert abs(g["clock"] - st.clock) <= 1e-15 * st.clock


def test_small_cut_60_steps_mixed(small_cut):
    """Mixed precision (stress, F, b^e in float32; the fracture test in
    float64 on the float32 stresses): every field within the mixed bound of
    the float64 oracle (measured: 2e-6) and the same MPs failed."""
    w, p, st = small_cut
    sim, _ = make_sim(w, precision="mixed")
    sim.init()
    sim.run(w.steps)
    sim.check_diag()
    g = sim.fields()
    assert np.array_equal(g["failed"], st.failed)
    errs = compare(gpu_fields(g, w.x_nodes, w.x_mp, p["T_r"]),
                   oracle_fields(st, w.x_nodes, w.x_mp, p["T_r"]))
    print("small cut, mixed, 60 steps:", json.dumps({k: float(v) for k, v in errs.items()}))
    bad = {k: v for k, v in errs.items() if not v < 1e-5}
    assert not bad, bad


def test_cutting_slab_runs_at_full_size():
    """The paper-size slab: 20 steps without a device failure; the clock and
    the lumped mass (failed MPs keep theirs) behave."""
    w = W.config_by_name("cutting_slab")
    sim, p = make_sim(w)
    sim.init()
    sim.run(20)
    code, _ = sim.check_diag()
    g = sim.fields()
    assert abs(g["clock"] - 20 * w.dt) < 1e-15 * 20 * w.dt
    assert abs(g["m"].sum() - w.mass_mp.sum()) < 1e-12 * w.mass_mp.sum()
    assert g["failed"].dtype == bool and np.all(g["sigma"][g["failed"]] == 0.0)
