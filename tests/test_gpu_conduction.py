"""Heat conduction through the LME gradients on the GPU against the oracle:
a bar at rest with a cosine temperature field (pure conduction), and the
small cut with plastic heating, fracture, the tool and erosion, with the
conductivity raised so that conduction moves heat within the run; float64
within 1e-10 for every field, mixed precision within 1e-5."""
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
MIXED_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _heat_fields(g, st):
    return (dict(q=g["q"], heat_h=g["heat_h"], heat_Q=g["heat_Q"]),
            dict(q=st.q, heat_h=st.heat_h, heat_Q=st.heat_Q))


def _bar_T0(xp):
    return 1.0 + 0.1 * np.cos(np.pi * xp[:, 0] / 20.0) + 0.02 * np.sin(np.pi * xp[:, 1] / 2.0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_heat_bar_matches_oracle(precision):
    w = W.heat_bar(n=(21, 3, 3), steps=200)
    p = W.params_from_workload(w)
    st = OST.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    st.T = _bar_T0(st.xp)
    OST.assemble(st, p)
    for _ in range(w.steps):
        OST.step(st, p)
    print(f"heat bar, {precision}, {w.n_mp} MPs", flush=True)
    sim, _ = make_sim(w, precision=precision)
    sim.init()
    sim.T.copy_(torch.from_numpy(_bar_T0(w.x_mp)))
    sim.refresh(rebuild=False)
    sim.run(w.steps)
    sim.check_diag()
    g = sim.fields()
    dT_gpu, dT_ref = g["T"] - 1.0, st.T - 1.0
    errs = {"dT": float(np.abs(dT_gpu - dT_ref).max() / np.abs(dT_ref).max())}
    a, b = _heat_fields(g, st)
    errs.update({k: float(v) for k, v in compare(a, b).items()})
    print(json.dumps(errs))
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    bad = {k: v for k, v in errs.items() if not v < tol}
    assert not bad, bad
    # total heat conserved on the GPU too (sum_I grad N_Ip = 0 holds to the
    # rounding of the stored grad N: float32 in the mixed mode)
    H0 = (w.mass_mp * _bar_T0(w.x_mp)).sum()
    tol_h = 1e-12 if precision == "fp64" else 1e-9
    assert abs((w.mass_mp * g["T"]).sum() - H0) <= tol_h * H0


def _cut_params(w):
    # Ti-alloy conductivity ~7 W/(m K) raised 300-fold: conduction then moves
    # heat over a few lattice spacings within the 60 steps
    return dict(kappa=2100.0)


@pytest.fixture(scope="module")
def oracle_cut():
    w = W.config_by_name("small_cut")
    p = W.params_from_workload(w, **_cut_params(w))
    st = OST.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    orig = np.arange(w.n_mp)
    for s in range(1, w.steps + 1):
        OST.step(st, p)
        if s in (30, 45):
            orig = orig[~st.failed]
            OST.erode(st, p)
    assert st.failed is not None and (st.T - p["T_r"]).max() > 1.0
    return w, p, st, orig


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_small_cut_with_conduction_matches_oracle(oracle_cut, precision):
    w, p, st, orig = oracle_cut
    print(f"small cut with conduction, {precision}", flush=True)
    sim, _ = make_sim(w, precision=precision, **_cut_params(w))
    sim.init()
    for s in range(1, w.steps + 1):
        sim.step()
        if s in (30, 45):
            sim.erode()
    sim.check_diag()
    g = sim.fields()
    assert sim.n_mp == st.xp.shape[0]
    assert np.array_equal(g["failed"], st.failed)
    if precision == "fp64":
        assert np.array_equal(g["idx"], st.idx)
    errs = compare(gpu_fields(g, w.x_nodes, w.x_mp[orig], p["T_r"]),
                   oracle_fields(st, w.x_nodes, w.x_mp[orig], p["T_r"]))
    a, b = _heat_fields(g, st)
    errs.update(compare(a, b))
    print(json.dumps({k: float(v) for k, v in errs.items()}))
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    bad = {k: v for k, v in errs.items() if not v < tol}
    assert not bad, bad


def test_conduction_needs_the_atomic_assembly():
    from paper_2206_08772_amd import _lib
    w = W.heat_bar(n=(5, 3, 3))
    sim, _ = make_sim(w, scatter="segmented")
    with pytest.raises(_lib.OtmError):
        sim.init()
