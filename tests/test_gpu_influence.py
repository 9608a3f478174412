"""Influence lists with large buckets.  The elastic cube's node lattice gets
extra MPs in part of its interior, so that the nodes there lie in the supports
of over 256 MPs (past what the bucket sort of the deterministic assembly holds
in registers; those buckets are ranked from memory) and the nodes around that
region in 160 to 320.  After one step (the stress is zero at t = 0) the
segmented assembly's mass and force must match the oracle, agree with the
atomic assembly, and repeat bit for bit."""
import dataclasses

import numpy as np
import pytest
import torch

import otm_workloads as W
from oracle import step as OST
from tests.gpu_common import make_sim, require_gpu
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def dense_cube():
    w = W.elastic_cube()
    rng = np.random.default_rng(11)
    extra = rng.uniform(2.0, 7.0, (750, 3))   # about the lattice's own MP density
    vol = np.concatenate([w.vol_mp, np.full(len(extra), 1.0 / 6.0)])
    return dataclasses.replace(w, name="dense_cube", x_mp=np.vstack([w.x_mp, extra]),
                               vol_mp=vol, mass_mp=w.material.rho0 * vol)


def _gpu_step(w, scatter):
    sim, _ = make_sim(w, scatter=scatter)
    sim.init()
    sim.step()
    sim.check_diag()
    torch.cuda.synchronize()
    f = sim.fields()
    return f["m"], f["f"]


def test_large_buckets_segmented_assembly(dense_cube):
    w = dense_cube
    p = W.params_from_workload(w)
    st = OST.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    OST.step(st, p)
    bucket = np.bincount(st.idx[:st.offsets[-1]], minlength=len(w.x_nodes))
    print(f"largest bucket {bucket.max()}, buckets over 256: {(bucket > 256).sum()}, "
          f"in (200, 256]: {((bucket > 200) & (bucket <= 256)).sum()}", flush=True)
    assert bucket.max() > 256 and ((bucket > 200) & (bucket <= 256)).any()
    m_ref, f_ref = st.m, st.f
    m_s1, f_s1 = _gpu_step(w, "segmented")
    m_s2, f_s2 = _gpu_step(w, "segmented")
    m_a, f_a = _gpu_step(w, "atomic")
    assert np.array_equal(m_s1, m_s2) and np.array_equal(f_s1, f_s2)
    for m, f in ((m_s1, f_s1), (m_a, f_a)):
        assert rel_err(m, m_ref) <= 1e-10
        assert rel_err(f, f_ref) <= 1e-10
    assert rel_err(f_s1, f_a) <= 1e-12
