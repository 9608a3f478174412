"""Parity of the stabilised step (Sec. 2.1, stabilised residual) with the
oracle, through the C ABI.  eps = mu h^2 changes the 100-step small-rod
trajectory by about 10 % against eps = 0, so a dropped or misplaced term
cannot pass."""
import json

import numpy as np
import pytest

import otm_workloads as W
from oracle import step as OST
from tests.gpu_common import make_sim, require_gpu
from tests.helpers import compare, gpu_fields, oracle_fields, rel_err

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _eps(w):
    mu = w.material.E / (2 * (1 + w.material.nu))
    return mu * w.h ** 2


def _oracle(w, steps, **over):
    p = W.params_from_workload(w, **over)
    st = OST.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    for _ in range(steps):
        OST.step(st, p)
    return st, p


def _gpu(w, steps, precision="fp64", scatter="atomic", **over):
    sim, p = make_sim(w, precision, scatter, **over)
    sim.init()
    sim.run(steps, rebuild_every=int(p["rebuild_every"]))
    sim.check_diag()
    return sim.fields(), sim


@pytest.fixture(scope="module")
def rod():
    w = W.config_by_name("small_rod")
    st, p = _oracle(w, 100, eps_stab=_eps(w))
    return w, st, p


@pytest.mark.parametrize("scatter", ["atomic", "segmented"])
def test_stabilised_small_rod_100_steps_fp64(rod, scatter):
    w, st, p = rod
    g, sim = _gpu(w, 100, scatter=scatter, eps_stab=p["eps_stab"])
    assert np.array_equal(g["offsets"], st.offsets) and np.array_equal(g["idx"], st.idx)
    errs = compare(gpu_fields(g, w.x_nodes, w.x_mp, p["T_r"]),
                   oracle_fields(st, w.x_nodes, w.x_mp, p["T_r"]))
    bad = {k: v for k, v in errs.items() if not v < FP64_TOL}
    assert not bad, bad
    # the history the last MP update left behind
    assert rel_err(sim.xp_prev.t().cpu().numpy() - w.x_mp, st.xp_prev - w.x_mp) < FP64_TOL
    dF = sim.dFm1.t().cpu().numpy().reshape(-1, 3, 3)
    assert rel_err(dF, st.dF - np.eye(3)) < FP64_TOL


def test_stabilised_small_rod_100_steps_mixed(rod):
    w, st, p = rod
    g, _ = _gpu(w, 100, precision="mixed", eps_stab=p["eps_stab"])
    errs = compare(gpu_fields(g, w.x_nodes, w.x_mp, p["T_r"]),
                   oracle_fields(st, w.x_nodes, w.x_mp, p["T_r"]))
    print("stabilised mixed-precision errors after 100 steps:", json.dumps(errs))
    bad = {k: v for k, v in errs.items() if not v < MIXED_TOL}
    assert not bad, bad


def test_stabilised_elastic_cube_10_steps_fp64():
    w = W.config_by_name("elastic_cube")
    st, p = _oracle(w, 10, eps_stab=_eps(w))
    g, _ = _gpu(w, 10, eps_stab=p["eps_stab"])
    errs = compare(gpu_fields(g, w.x_nodes, w.x_mp, p["T_r"]),
                   oracle_fields(st, w.x_nodes, w.x_mp, p["T_r"]))
    bad = {k: v for k, v in errs.items() if not v < FP64_TOL}
    assert not bad, bad


def test_the_term_changes_the_trajectory(rod):
    w, st, p = rod
    g0, _ = _gpu(w, 100)
    u_eps = st.x - w.x_nodes
    assert rel_err(g0["x"] - w.x_nodes, u_eps) > 1e-2
