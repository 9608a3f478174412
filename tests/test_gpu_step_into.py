"""otm_step_into against otm_step: the same trajectory, with the lists and
shape functions of every step left intact in the arrays the step moved away
from (what the checkpointed adjoint's tape relies on)."""
import numpy as np
import pytest

import otm_workloads as W
from tests.gpu_common import make_sim, require_gpu
from tests.helpers import rel_err

pytestmark = pytest.mark.gpu

FIELDS = ("x", "du", "m", "f", "xp", "vol", "sigma", "epsbar", "T", "N", "dN", "lam",
          "offsets", "idx")
LISTS = ("offsets", "idx", "N", "dN")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _lists_like(sim):
    return {k: getattr(sim, k).clone().fill_(0) for k in LISTS}


def _host_lists(sim):
    return {k: getattr(sim, k).cpu().numpy().copy() for k in LISTS}


@pytest.mark.parametrize("scatter,rebuild_every", [("segmented", 1), ("atomic", 1),
                                                   ("segmented", 3)])
def test_step_into_matches_step(scatter, rebuild_every):
    w = W.config_by_name("small_rod")
    ref, _ = make_sim(w, scatter=scatter)
    sim, _ = make_sim(w, scatter=scatter)
    ref.init()
    sim.init()
    # three list sets in rotation: the state's own, then two spares
    sets = [{k: getattr(sim, k) for k in LISTS}, _lists_like(sim), _lists_like(sim)]
    for n in range(1, 8):
        rebuild = n % rebuild_every == 0
        before = _host_lists(sim)
        old = {k: getattr(sim, k) for k in LISTS}
        assert old["N"].data_ptr() == sets[(n - 1) % 3]["N"].data_ptr()
        target = sets[n % 3]
        ref.step(rebuild=rebuild)
        sim.step_into(target, rebuild=rebuild)
        assert all(getattr(sim, k).data_ptr() == target[k].data_ptr() for k in LISTS)
        # the arrays given up still hold the previous step's lists
        after_old = {k: old[k].cpu().numpy() for k in LISTS}
        for k in LISTS:
            assert np.array_equal(after_old[k], before[k]), (n, k)
        a, b = ref.fields(), sim.fields()
        for k in FIELDS:
            if scatter == "segmented" or k in ("offsets", "idx"):
                assert np.array_equal(a[k], b[k]), (n, k)
            else:
                x0 = {"x": w.x_nodes, "xp": w.x_mp}.get(k, 0.0)
                assert rel_err(b[k] - x0, a[k] - x0) < 1e-11, (n, k)
    ref.check_diag()
    sim.check_diag()
