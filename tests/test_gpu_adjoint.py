"""Adjoint of the step (checkpointed rollout) against the oracle's
complex-step gradient and against central finite differences."""
import numpy as np
import pytest
import torch

import otm_workloads as W
from oracle import gradient as OG
from tests.gpu_common import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _problem(w, p, steps, every):
    speed = float(np.abs(w.v0_nodes).max())
    return dict(x_nodes=w.x_nodes, x_mp=w.x_mp, vol_mp=w.vol_mp, mass_mp=w.mass_mp,
                v0_unit=w.v0_nodes / speed, params=p, steps=steps, every=every), speed


def _gpu_grad(problem, speed, p, target):
    from paper_2206_08772_amd.adjoint import OTMRollout
    theta = torch.tensor([p["A"], p["B"], p["n"]], dtype=torch.float64, requires_grad=True)
    sp = torch.tensor(speed, dtype=torch.float64, requires_grad=True)
    x = OTMRollout.apply(theta, sp, problem)
    tgt = torch.as_tensor(target, device=x.device)
    loss = 0.5 * ((x - tgt) ** 2).sum()
    loss.backward()
    return float(loss), theta.grad.cpu().numpy(), float(sp.grad)


@pytest.mark.parametrize("radius_scale", [1.0, 1.15])
def test_adjoint_matches_complex_step_oracle(radius_scale):
    """Tiny J2/JC rod, 8 steps, checkpoints every 3: gradients of the final
    position mismatch with respect to A, B, n and the impact speed.  The wider
    search radius gives supports of 20 to 45 nodes, so the MPs above 40 go
    through the adjoint's long-support launch."""
    w = W.taylor_rod(h=0.8e-3, seed=5, radius=2.4e-3, length=6.4e-3, steps=8, name="tiny_rod")
    p = W.params_from_workload(w)
    r = p["r_list"] * radius_scale
    p = dict(p, r_list=r, cell_size=max(p["cell_size"], r))
    steps = 8
    lists, _ = OG.nominal_lists(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, steps)
    K = np.concatenate([np.diff(off) for off, _ in lists[1:]])
    assert K.max() <= 48
    if radius_scale > 1:
        assert (K > 40).sum() > 50
    # target: the oracle with perturbed hardening constants
    pt = dict(p, A=p["A"] * 1.05, B=p["B"] * 0.95, n=p["n"] + 0.02)
    tgt_lists, st_t = OG.nominal_lists(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, pt,
                                       steps)
    target = st_t.x
    ref = OG.complex_step_gradient(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, steps,
                                   lists, target)
    problem, speed = _problem(w, p, steps, every=3)
    loss, gth, gsp = _gpu_grad(problem, speed, p, target)
    for k, name in enumerate(("A", "B", "n")):
        assert abs(gth[k] - ref[name]) <= 1e-6 * abs(ref[name]), (name, gth[k], ref[name])
    assert abs(gsp - ref["speed"]) <= 1e-6 * abs(ref["speed"]), (gsp, ref["speed"])


def _run(w, p, steps, speed, unit, lists=None, record=None):
    """GPU rollout.  With ``lists`` the support lists of step n are replayed
    (frozen to a nominal trajectory); with ``record`` they are stored."""
    from paper_2206_08772_amd.sim import Sim
    sim = Sim(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, speed * unit, p)
    sim.init()
    for n in range(1, steps + 1):
        if lists is None:
            sim.step()
        else:
            sim.step(rebuild=False)
            off, idx = lists[n]
            sim.offsets.copy_(off)
            sim.idx[:idx.numel()].copy_(idx)
            sim.refresh(rebuild=False)
        if record is not None:
            P = int(sim.offsets[-1])
            record.append((sim.offsets.clone(), sim.idx[:P].clone()))
    sim.check_diag()
    return sim.x.t().contiguous()


def test_adjoint_against_finite_differences_adjoint_rod():
    """268k MPs, 200 steps, checkpoints every 20; central differences with a
    relative step of 1e-6 on rollouts whose support lists are frozen to the
    nominal trajectory; agreement to 1e-4."""
    w = W.config_by_name("adjoint_rod")
    p = W.params_from_workload(w)
    steps = w.steps
    problem, speed = _problem(w, p, steps, every=20)
    unit = problem["v0_unit"]
    pt = dict(p, A=p["A"] * 1.05, B=p["B"] * 0.95, n=p["n"] + 0.02)
    target = _run(w, pt, steps, speed, unit)
    lists = [None]
    _run(w, p, steps, speed, unit, record=lists)
    loss, gth, gsp = _gpu_grad(problem, speed, p, target)

    def L(pp, sp):
        x = _run(w, pp, steps, sp, unit, lists=lists)
        return 0.5 * float(((x - target) ** 2).sum())

    rel = {}
    for k, name in enumerate(("A", "B", "n")):
        e = 1e-6 * abs(p[name])
        fd = (L(dict(p, **{name: p[name] + e}), speed) - L(dict(p, **{name: p[name] - e}), speed)) \
            / (2 * e)
        rel[name] = abs(gth[k] - fd) / abs(fd)
    e = 1e-6 * speed
    fd = (L(p, speed + e) - L(p, speed - e)) / (2 * e)
    rel["speed"] = abs(gsp - fd) / abs(fd)
    print("adjoint vs central differences (relative):", rel)
    assert all(v <= 1e-4 for v in rel.values()), rel
