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


def _flag(code):
    return 1 << (-code - 1)


def test_nonfinite_stress_state_is_reported_at_its_mp():
    """NaN written from the host into b^e of one MP: the MP pass returns a
    non-finite stress for that MP alone (every loop of the return map is
    bounded, so the kernels finish), which is reported with its index."""
    from paper_2206_08772_amd import _lib
    w = W.config_by_name("small_rod")
    sim, p = make_sim(w, scatter="segmented")
    sim.init()
    for _ in range(3):
        sim.step()
    assert sim.check_diag()[0] == 0
    k = 1234
    sim.bed[:, k] = float("nan")
    sim.step(rebuild=False)
    code, d = sim.check_diag(raise_on_error=False)
    assert d.flags & _flag(_lib.OTM_ERR_NONFINITE)
    assert d.n_nonfinite == 1 and d.first_nonfinite == k
    assert torch.isnan(sim.sigma[:, k]).all()
    assert torch.isfinite(sim.sigma[:, :k]).all() and torch.isfinite(sim.sigma[:, k + 1:]).all()


def test_nonfinite_node_force_is_reported_at_the_node_and_its_mps():
    """NaN written into the force of one node I: the node update reports the
    node (index n_mp + I) and the MP pass every MP whose support holds I
    (their positions gather the NaN); the smallest of those MPs is the first
    index."""
    from paper_2206_08772_amd import _lib
    w = W.config_by_name("small_rod")
    sim, p = make_sim(w, scatter="segmented")
    sim.init()
    sim.step()
    assert sim.check_diag()[0] == 0
    g = sim.fields()
    I = int(g["idx"][g["offsets"][500]])           # a node of MP 500's support
    mp_of_pair = np.repeat(np.arange(sim.n_mp), np.diff(g["offsets"]))
    users = np.unique(mp_of_pair[g["idx"] == I])
    assert users.size > 5
    sim.f[1, I] = float("nan")
    sim.step(rebuild=False)
    code, d = sim.check_diag(raise_on_error=False)
    assert d.flags & _flag(_lib.OTM_ERR_NONFINITE)
    assert d.first_nonfinite == users.min()
    assert d.n_nonfinite == 1 + users.size
    assert torch.isnan(sim.x[:, I]).any()


def test_return_map_non_convergence_is_reported():
    """rm_max_iter = 1 on a step with plastic flow: the return map of the
    yielding MPs stops unconverged.  Two bit-identical runs (segmented
    assembly) reach the same state; the next step with the normal limit
    tells which MPs yield, and the capped step reports those, with the first
    index among them."""
    from paper_2206_08772_amd import _lib
    w = W.config_by_name("small_rod")
    a, _ = make_sim(w, scatter="segmented")
    b, _ = make_sim(w, scatter="segmented")
    for s in (a, b):
        s.init()
        s.run(6)
        assert s.check_diag()[0] == 0
    eb0 = a.epsbar.cpu().numpy().copy()
    a.step()
    plastic = np.nonzero(a.epsbar.cpu().numpy() > eb0)[0]
    assert plastic.size > 20
    b.p.rm_max_iter = 1
    b.step()
    code, d = b.check_diag(raise_on_error=False)
    assert code == _lib.OTM_ERR_RM_NOCONV
    assert d.first_rm_noconv in set(plastic.tolist())
    assert 0.9 * plastic.size <= d.n_rm_noconv <= plastic.size
