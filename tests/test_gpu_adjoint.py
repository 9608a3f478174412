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


JC = ("A", "B", "n", "C", "m")


def _gpu_grad(problem, speed, p, target):
    from paper_2206_08772_amd.adjoint import OTMRollout
    theta = torch.tensor([p[k] for k in JC], dtype=torch.float64, requires_grad=True)
    sp = torch.tensor(speed, dtype=torch.float64, requires_grad=True)
    x = OTMRollout.apply(theta, sp, problem)
    tgt = torch.as_tensor(target, device=x.device)
    loss = 0.5 * ((x - tgt) ** 2).sum()
    loss.backward()
    return loss.item(), theta.grad.cpu().numpy(), sp.grad.item()


@pytest.mark.parametrize("radius_scale", [1.0, 1.15])
def test_adjoint_matches_complex_step_oracle(radius_scale):
    """Tiny J2/JC rod, 8 steps, checkpoints every 3: gradients of the final
    position mismatch with respect to A, B, n, C, m, the impact speed and,
    through OTMRolloutField, along a random initial velocity field.  The wider
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
    d = np.random.default_rng(3).standard_normal(w.v0_nodes.shape) * np.abs(w.v0_nodes).max()
    ref = OG.complex_step_gradient(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, steps,
                                   lists, target, params=JC, v0_dirs=(d,))
    problem, speed = _problem(w, p, steps, every=3)
    loss, gth, gsp = _gpu_grad(problem, speed, p, target)
    for k, name in enumerate(JC):
        assert abs(gth[k] - ref[name]) <= 1e-6 * abs(ref[name]), (name, gth[k], ref[name])
    assert abs(gsp - ref["speed"]) <= 1e-6 * abs(ref["speed"]), (gsp, ref["speed"])
    # the per-node initial-velocity gradient, along the random field d
    from paper_2206_08772_amd.adjoint import OTMRolloutField
    theta = torch.tensor([p[k] for k in JC], dtype=torch.float64, requires_grad=True)
    v0 = torch.tensor(w.v0_nodes, dtype=torch.float64, requires_grad=True)
    x = OTMRolloutField.apply(theta, v0, problem)
    tgt = torch.as_tensor(target, device=x.device)
    (0.5 * ((x - tgt) ** 2).sum()).backward()
    assert v0.grad.shape == w.v0_nodes.shape
    gdir = float((v0.grad.numpy() * d).sum())
    assert abs(gdir - ref[("v0", 0)]) <= 1e-6 * abs(ref[("v0", 0)]), (gdir, ref[("v0", 0)])
    assert np.allclose(theta.grad.numpy(), gth, rtol=1e-12, atol=0)


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
    """268k MPs, 200 steps, checkpoints every 20: the gradients by A, B, n,
    C, m and the impact speed against central differences (relative step
    1e-6, 1e-4 for C and m) on rollouts whose support lists are frozen to the
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
    for k, name in enumerate(JC):
        # C and m move the loss by little: a larger step keeps their
        # differences well above round-off
        e = (1e-6 if name in ("A", "B", "n") else 1e-4) * abs(p[name])
        fd = (L(dict(p, **{name: p[name] + e}), speed) - L(dict(p, **{name: p[name] - e}), speed)) \
            / (2 * e)
        rel[name] = abs(gth[k] - fd) / abs(fd)
    e = 1e-6 * speed
    fd = (L(p, speed + e) - L(p, speed - e)) / (2 * e)
    rel["speed"] = abs(gsp - fd) / abs(fd)
    print("adjoint vs central differences (relative):", rel)
    assert all(v <= 1e-4 for v in rel.values()), rel


# ------------------------------------------------------ dot-product test
SYM = ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2))   # stored order of b^e and sigma


def _gpu_layout(field, a):
    """Oracle array -> the library's device layout (as a host array)."""
    a = np.asarray(a, np.float64)
    if field in ("x", "du", "xp", "lam", "f"):
        return np.ascontiguousarray(a.T)
    if field == "F":
        return np.ascontiguousarray((a - np.eye(3)).reshape(-1, 9).T)
    if field == "be":
        a = a - np.eye(3)
    if field in ("be", "sigma"):
        return np.stack([a[:, i, j] for i, j in SYM])
    if field == "dN":
        return np.ascontiguousarray(a.T)
    return a


def _tangent_layout(field, a):
    """A tangent (or derivative) of an oracle field in the stored components
    the adjoint is taken with respect to."""
    a = np.asarray(a, np.float64)
    if field in ("x", "du", "dN"):
        return np.ascontiguousarray(a.T)
    if field == "F":
        return np.ascontiguousarray(a.reshape(-1, 9).T)
    if field in ("be", "sigma"):
        return np.stack([a[:, i, j] for i, j in SYM])
    return a


BAR_OF = {"x": "x", "du": "du", "vol": "vol", "F": "Fd", "be": "bed", "epsbar": "epsbar",
          "T": "T", "sigma": "sigma", "N": "N", "dN": "dN"}


def _tape(st, cap):
    from paper_2206_08772_amd._lib import Tape
    from paper_2206_08772_amd.sim import _ptr
    keep = {}
    t = Tape()
    t.n_nodes, t.n_mp, t.pair_stride = st.x.shape[0], st.xp.shape[0], cap
    for k, name in (("x", "x"), ("du", "du"), ("m", "m"), ("f", "f"), ("xp", "xp"),
                    ("vol", "vol"), ("lam", "lam"), ("F", "Fd"), ("be", "bed"),
                    ("epsbar", "epsbar"), ("T", "T"), ("sigma", "sigma")):
        keep[name] = torch.from_numpy(_gpu_layout(k, getattr(st, k))).cuda()
    P = st.idx.shape[0]
    N = np.zeros(cap)
    N[:P] = st.N
    dN = np.zeros((3, cap))
    dN[:, :P] = st.dN.T
    keep["N"] = torch.from_numpy(N).cuda()
    keep["dN"] = torch.from_numpy(dN).cuda()
    keep["offsets"] = torch.from_numpy(np.asarray(st.offsets, np.int64)).cuda()
    idx = np.zeros(cap, np.int32)
    idx[:P] = st.idx
    keep["idx"] = torch.from_numpy(idx).cuda()
    for name in ("x", "du", "m", "f", "xp", "vol", "lam", "Fd", "bed", "epsbar", "T", "sigma",
                 "N", "dN"):
        setattr(t, name, _ptr(keep[name]).value)
    t.nbr_offsets = _ptr(keep["offsets"]).value
    t.nbr_idx = _ptr(keep["idx"]).value
    return t, keep


def test_adjoint_step_dot_products_against_oracle_jvp():
    """For one step of the tiny rod (state after 4 steps: plastic flow, heating
    and wall contact under way), <bar_n, delta> from otm_step_adjoint equals
    <bar_{n+1}, J delta> from the oracle's complex-step derivative of the
    one-step map, for every (input field, output field) block: a seeded
    adjoint on one output field at a time, a seeded tangent of one input field
    at a time.  The hardening-constant gradient is checked the same way."""
    import ctypes as C
    from oracle import step as OS
    from paper_2206_08772_amd import _lib
    from paper_2206_08772_amd.adjoint import Bars
    from paper_2206_08772_amd.sim import _ptr, _stream, make_params, new_diag, read_diag
    from tests.helpers import step_directions
    w = W.taylor_rod(h=0.8e-3, seed=5, radius=2.4e-3, length=6.4e-3, steps=8, name="tiny_rod")
    p = W.params_from_workload(w)
    lists, _ = OG.nominal_lists(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, 5)
    st = OG.rollout(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, 4, lists)
    s1 = OG.step_map(st, p, lists[5])
    OS.assemble(s1, p)
    assert st.epsbar.max() > 0
    dirs = step_directions(st, np.random.default_rng(1))
    jvp = {k: OG.step_jvp(st, p, lists[5], direction={k: dirs[k]}) for k in OG.STEP_FIELDS}
    jvp_th = {k: OG.step_jvp(st, p, lists[5], param=k) for k in JC}

    L = _lib.lib()
    nn, nm = st.x.shape[0], st.xp.shape[0]
    cap = max(st.idx.shape[0], s1.idx.shape[0])
    t0, keep0 = _tape(st, cap)
    t1, keep1 = _tape(s1, cap)
    mass = torch.from_numpy(np.asarray(w.mass_mp, np.float64)).cuda()
    pp = make_params(p)
    ws_bytes = int(L.otm_adjoint_workspace_bytes(nn, nm))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    diag = new_diag(torch.device("cuda"))
    rng = np.random.default_rng(2)
    P1 = s1.idx.shape[0]
    worst = 0.0
    for o in OG.STEP_FIELDS:
        nxt, cur = Bars(nn, nm, cap, "cuda"), Bars(nn, nm, cap, "cuda")
        ref = _tangent_layout(o, jvp[o][o])          # shape of the stored output field
        sbar = rng.standard_normal(ref.shape)        # pairs of step n+1 only
        tgt = getattr(nxt, BAR_OF[o])
        if o in ("N", "dN"):
            tgt[..., :P1].copy_(torch.from_numpy(np.ascontiguousarray(sbar[..., :P1])))
        else:
            tgt.copy_(torch.from_numpy(sbar))
        theta = torch.zeros(5, dtype=torch.float64, device="cuda")
        bn, bc = nxt.struct(), cur.struct()
        _lib.check(L.otm_step_adjoint(C.byref(t0), C.byref(t1), C.byref(pp), p["dt"], _ptr(mass),
                                      C.byref(bn), C.byref(bc), _ptr(theta), _ptr(ws), ws_bytes,
                                      _ptr(diag), _stream()), "otm_step_adjoint")
        torch.cuda.synchronize()
        P0 = st.idx.shape[0]
        scales, rows = [], []
        for i in OG.STEP_FIELDS:
            bar_i = getattr(cur, BAR_OF[i]).cpu().numpy()
            if i in ("N", "dN"):
                bar_i = bar_i[..., :P0]
            delta = _tangent_layout(i, dirs[i])
            lhs = float((bar_i * delta).sum())
            jo = _tangent_layout(o, jvp[i][o])
            rhs = float((sbar * jo).sum())
            scale = float(np.abs(sbar * jo).sum())
            rows.append((i, lhs, rhs, scale))
            scales.append(scale)
        top = max(scales)
        for i, lhs, rhs, scale in rows:
            tol = 1e-8 * scale + 1e-12 * top
            assert abs(lhs - rhs) <= tol, (o, i, lhs, rhs, scale)
            if scale > 0:
                worst = max(worst, abs(lhs - rhs) / scale)
        th = theta.cpu().numpy()
        for k, name in enumerate(JC):
            jo = _tangent_layout(o, jvp_th[name][o])
            rhs = float((sbar * jo).sum())
            scale = float(np.abs(sbar * jo).sum())
            assert abs(th[k] - rhs) <= 1e-8 * scale, (o, name, th[k], rhs, scale)
    code, _ = read_diag(diag)
    assert code == _lib.OTM_OK
    print(f"adjoint dot products: worst |<bar_n, d> - <bar_n+1, J d>| / scale = {worst:.2e}")

