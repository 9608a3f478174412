"""Save and resume: a run saved after some steps and resumed in a fresh
simulation continues exactly as the uninterrupted run (segmented assembly,
so bit for bit), with the stabilisation history and with the chip-formation
state (failure flags, tangential gaps, tool clock)."""
import numpy as np
import pytest

import otm_workloads as W
from tests.gpu_common import make_sim, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _eps(w):
    return w.material.E / (2 * (1 + w.material.nu)) * w.h ** 2


@pytest.mark.parametrize("name", ["small_rod", "small_cut"])
def test_resume_continues_bit_for_bit(name, tmp_path):
    w = W.config_by_name(name)
    over = {"eps_stab": _eps(w)} if name == "small_rod" else {}
    a, _ = make_sim(w, scatter="segmented", **over)
    a.init()
    a.run(30)
    path = tmp_path / "state.pt"
    a.save(path)
    a.run(15)
    b, _ = make_sim(w, scatter="segmented", **over)
    b.load(path)
    assert b.n == 30
    b.run(15)
    fa, fb = a.fields(), b.fields()
    keys = ["x", "du", "m", "f", "xp", "vol", "sigma", "epsbar", "T", "N", "dN", "lam",
            "offsets", "idx"] + (["failed", "gT", "clock"] if name == "small_cut" else [])
    for k in keys:
        assert np.array_equal(np.asarray(fa[k]), np.asarray(fb[k])), k
    if name == "small_rod":
        assert np.array_equal(a.xp_prev.cpu().numpy(), b.xp_prev.cpu().numpy())
    a.check_diag()
    b.check_diag()


def test_resume_between_list_rebuilds_segmented():
    """Lists with a skin (radius r + 0.1 h) rebuilt every 10 steps, saved at
    step 15: the resumed run keeps the saved lists (not those of a search
    at the saved positions) and the influence lists built from them, and continues bit for bit through the rebuilds at 20 and 30."""
    w = W.config_by_name("small_rod")
    r = w.r_list + 0.1 * w.h
    over = dict(r_list=r, cell_size=r * 1.0001, rebuild_every=10)
    a, _ = make_sim(w, scatter="segmented", **over)
    a.init()
    a.run(15, rebuild_every=10)
    d = a.state_dict()
    a.run(20, rebuild_every=10)
    b, _ = make_sim(w, scatter="segmented", **over)
    b.load_state_dict(d)
    assert b.n == 15
    b.run(20, rebuild_every=10)
    fa, fb = a.fields(), b.fields()
    for k in ["x", "du", "m", "f", "xp", "vol", "sigma", "epsbar", "T", "N", "dN", "lam",
              "offsets", "idx"]:
        assert np.array_equal(np.asarray(fa[k]), np.asarray(fb[k])), k
    a.check_diag()
    b.check_diag()
