"""Device-side failure reporting (forced from the host; every kernel still
finishes normally)."""
import numpy as np
import pytest
import torch

import otm_workloads as W
from tests.gpu_common import make_sim, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_pair_capacity_overflow_is_reported_and_recoverable():
    from paper_2206_08772_amd import _lib
    w = W.config_by_name("small_rod")
    sim, p = make_sim(w)
    sim.init()
    code, d = sim.check_diag()
    P0 = d.pairs_needed
    # a larger search radius needs more pairs than the buffer holds
    sim.p.r_list *= 1.3
    sim.p.cell_size *= 1.3
    sim.refresh(rebuild=True)
    code, d = sim.check_diag(raise_on_error=False)
    assert code == _lib.OTM_ERR_CAPACITY
    assert d.pairs_needed > sim.cap > P0
    # after the radius is restored the lists fit again
    from paper_2206_08772_amd.sim import new_diag
    sim.diag = new_diag(sim.device)
    sim.p.r_list /= 1.3
    sim.p.cell_size /= 1.3
    sim.refresh(rebuild=True)
    assert sim.check_diag()[0] == 0


def test_inverted_material_points_are_reported():
    from paper_2206_08772_amd import _lib
    w = W.elastic_cube(n=4)
    sim, p = make_sim(w)
    sim.init()
    torch.cuda.synchronize()
    # prescribe du = -2.5 (x - c): dF = -1.5 * 1, det < 0 everywhere
    c = sim.x.mean(dim=1, keepdim=True)
    sim.du.copy_(-2.5 * (sim.x - c))
    sim.f.zero_()
    sim.step(rebuild=False)
    code, d = sim.check_diag(raise_on_error=False)
    assert d.flags & (1 << (-_lib.OTM_ERR_INVERTED - 1))
    assert d.n_inverted == w.n_mp and d.first_inverted == 0
