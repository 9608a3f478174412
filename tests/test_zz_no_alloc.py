"""otm_step_noalloc (the step with the library's static device scratch instead
of a caller workspace) against otm_step, through the C ABI: the paper-size
rod (27,840 MPs) and then the smaller rod (2,304 MPs) on the same device
scratch, segmented assembly bit for bit and atomic assembly to round-off,
with lists rebuilt every step and once carried over (rebuild = 0) right
after the larger state used the scratch."""
import ctypes as C

import numpy as np
import pytest

import otm_workloads as W
from tests.gpu_common import make_sim, require_gpu
from tests.helpers import compare, gpu_fields

pytestmark = pytest.mark.gpu

STEPS = 3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _noalloc_step(sim, rebuild):
    from paper_2206_08772_amd import _lib
    from paper_2206_08772_amd.sim import _ptr, _stream
    _lib.check(_lib.lib().otm_step_noalloc(C.byref(sim.st), C.byref(sim.p), sim.dt,
                                           1 if rebuild else 0, sim.mode, _ptr(sim.diag),
                                           _stream()), "otm_step_noalloc")
    sim.n += 1


def _fields(sim, w):
    sim.check_diag()
    g = sim.fields()
    out = gpu_fields(g, w.x_nodes, w.x_mp, 0.0)
    out["idx"] = g["idx"]
    out["offsets"] = g["offsets"]
    return out


@pytest.mark.parametrize("scatter", ["segmented", "atomic"])
def test_noalloc_step_matches_otm_step(scatter):
    from paper_2206_08772_amd import _lib
    for name in ("paper_rod", "small_rod"):       # the second call is the smaller input
        w = W.config_by_name(name)
        print(f"noalloc vs otm_step: {name}, {scatter}, {w.x_mp.shape[0]} MPs", flush=True)
        ref, _ = make_sim(w, scatter=scatter)
        got, _ = make_sim(w, scatter=scatter)
        assert got.cap == ref.cap
        ws_need = int(_lib.lib().otm_workspace_bytes(got.n_nodes, got.n_mp, got.cap))
        assert ws_need <= _lib.OTM_STATIC_SCRATCH_BYTES
        ref.init()
        got.init()
        for s in range(STEPS):
            rebuild = s != 0          # first step: lists of t = 0 carried over
            ref.step(rebuild=rebuild)
            _noalloc_step(got, rebuild)
        a, b = _fields(got, w), _fields(ref, w)
        assert np.array_equal(a["offsets"], b["offsets"]) and np.array_equal(a["idx"], b["idx"])
        if scatter == "segmented":
            for k in b:
                assert np.array_equal(a[k], b[k]), k
        else:
            errs = compare(a, b)
            bad = {k: v for k, v in errs.items() if not v <= 1e-12}
            assert not bad, bad
