"""Set-up shared by the GPU tests: the library must be built and loadable,
and a HIP device must be present (no fallback of any kind)."""
import numpy as np
import torch


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2206_08772_amd import _lib
    _lib.lib()   # raises if libotm.so is missing


def make_sim(w, precision="fp64", scatter="atomic", **over):
    import otm_workloads
    from paper_2206_08772_amd.sim import Sim
    p = otm_workloads.params_from_workload(w, **over)
    sim = Sim(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, precision=precision,
              scatter=scatter)
    return sim, p


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float64).T)).cuda()
