"""Pins of the oracle's erosion (removal of failed MPs, then a refresh of the
lists, shape functions, mass and force): against the step's own refresh when
nothing failed, against mass bookkeeping (the shape functions are a
partition of unity, so the lumped nodal masses sum to the mass of the MPs
that remain), against a body built from scratch out of the survivors, and
the degenerate case of a body that fails entirely."""
import numpy as np
import pytest

import otm_workloads as W
from oracle import step as OST
from tests.helpers import rel_err


@pytest.fixture(scope="module")
def cut():
    w = W.config_by_name("small_cut")
    p = W.params_from_workload(w)
    st = OST.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    early = None
    for s in range(45):
        OST.step(st, p)
        if s + 1 == 10:
            early = st.copy()
    assert not early.failed.any() and st.failed.sum() > 10
    return w, p, early, st


def test_erode_with_nothing_failed_is_the_steps_refresh(cut):
    w, p, early, _ = cut
    st = early.copy()
    assert OST.erode(st, p) == 0
    assert np.array_equal(st.offsets, early.offsets) and np.array_equal(st.idx, early.idx)
    for k in ("N", "dN", "m", "f", "lam"):
        assert rel_err(getattr(st, k), getattr(early, k)) < 1e-12, k


def test_erode_removes_exactly_the_failed_mass(cut):
    w, p, _, late = cut
    st = late.copy()
    n0, nf = st.xp.shape[0], int(late.failed.sum())
    assert abs(late.m.sum() - late.mass.sum()) < 1e-13 * late.mass.sum()
    assert OST.erode(st, p) == nf
    assert st.xp.shape[0] == n0 - nf and not st.failed.any()
    assert st.offsets.shape[0] == n0 - nf + 1 and st.idx.shape[0] == st.offsets[-1]
    lost = late.mass[late.failed].sum()
    assert abs((late.m.sum() - st.m.sum()) - lost) < 1e-12 * late.mass.sum()
    assert np.abs(st.f).max() > 0


def test_erode_matches_a_body_built_from_the_survivors(cut):
    """Lists, shape functions and lumped mass after erosion equal those of a
    fresh start on the survivors' positions and masses (the Newton solve
    starts there from zero multipliers instead of warm, hence 1e-11)."""
    w, p, _, late = cut
    st = late.copy()
    OST.erode(st, p)
    keep = ~late.failed
    fresh = OST.init_state(late.x, late.xp[keep], late.vol[keep], late.mass[keep],
                           np.zeros_like(late.x), p)
    assert np.array_equal(st.offsets, fresh.offsets) and np.array_equal(st.idx, fresh.idx)
    assert rel_err(st.N, fresh.N) < 1e-11 and rel_err(st.m, fresh.m) < 1e-11
    assert rel_err(st.dN, fresh.dN) < 1e-10


def test_erode_a_body_that_failed_entirely(cut):
    w, p, _, late = cut
    st = late.copy()
    st.failed[:] = True
    assert OST.erode(st, p) == late.xp.shape[0]
    assert st.xp.shape == (0, 3) and st.offsets.tolist() == [0]
    assert not st.m.any() and not st.f.any()
