"""Pin of the oracle's complex-step gradient: central finite differences of
the real oracle on the same frozen lists (relative step 1e-6; agreement to
1e-4, the accuracy of the differences: measured 1e-5 for B)."""
import numpy as np
import pytest

import otm_workloads as W
from oracle import gradient as OG


@pytest.fixture(scope="module")
def setup():
    w = W.taylor_rod(h=0.8e-3, seed=5, radius=2.4e-3, length=6.4e-3, steps=8, name="tiny_rod")
    p = W.params_from_workload(w)
    steps = 8
    lists, st = OG.nominal_lists(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, steps)
    rng = np.random.default_rng(0)
    target = st.x + 1e-6 * rng.standard_normal(st.x.shape)
    return w, p, steps, lists, target, st


def test_complex_rollout_primal_matches_real(setup):
    w, p, steps, lists, target, st = setup
    stc = OG.rollout(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, steps, lists,
                     complex_step=True)
    assert st.epsbar.max() > 0                      # plastic flow in the run
    u = st.x - w.x_nodes
    assert np.abs(stc.x.real - st.x).max() < 1e-12 * np.abs(u).max()
    assert np.abs(stc.x.imag).max() == 0.0


def test_complex_step_matches_central_differences(setup):
    w, p, steps, lists, target, st = setup
    d = np.random.default_rng(3).standard_normal(w.v0_nodes.shape) * np.abs(w.v0_nodes).max()
    g = OG.complex_step_gradient(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, steps,
                                 lists, target, params=("A", "B", "n", "C", "m"), v0_dirs=(d,))
    for name in ("A", "B", "n", "C", "m"):
        # C and m move the loss by little (rate factor and the small heating
        # of 8 steps): a larger step keeps their differences above round-off
        e = (1e-6 if name in ("A", "B", "n") else 1e-4) * abs(p[name])
        lp = OG.loss(OG.rollout(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes,
                                dict(p, **{name: p[name] + e}), steps, lists), target)
        lm = OG.loss(OG.rollout(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes,
                                dict(p, **{name: p[name] - e}), steps, lists), target)
        fd = (lp - lm) / (2 * e)
        assert abs(g[name] - fd) <= 1e-4 * abs(fd), (name, g[name], fd)
    s = np.abs(w.v0_nodes).max()
    e = 1e-6 * s
    lp = OG.loss(OG.rollout(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes * (1 + e / s), p,
                            steps, lists), target)
    lm = OG.loss(OG.rollout(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes * (1 - e / s), p,
                            steps, lists), target)
    fd = (lp - lm) / (2 * e)
    assert abs(g["speed"] - fd) <= 1e-4 * abs(fd), (g["speed"], fd)
    # along a random initial velocity field (per-node gradient)
    e = 1e-6
    lp = OG.loss(OG.rollout(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes + e * d, p,
                            steps, lists), target)
    lm = OG.loss(OG.rollout(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes - e * d, p,
                            steps, lists), target)
    fd = (lp - lm) / (2 * e)
    assert abs(g[("v0", 0)] - fd) <= 1e-4 * abs(fd), (g[("v0", 0)], fd)


@pytest.fixture(scope="module")
def one_step():
    """State of the tiny rod after 4 steps (plastic flow and heating under way)
    and the nominal lists of step 5."""
    w = W.taylor_rod(h=0.8e-3, seed=5, radius=2.4e-3, length=6.4e-3, steps=8, name="tiny_rod")
    p = W.params_from_workload(w)
    lists, _ = OG.nominal_lists(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, 5)
    st = OG.rollout(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, 4, lists)
    return st, p, lists[5]


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
@pytest.mark.parametrize("field", OG.STEP_FIELDS + ("A", "B", "n", "C", "m"))
def test_step_jvp_matches_central_differences(one_step, field):
    """The complex-step derivative of the one-step map along a seeded direction
    of each state field (and by each hardening constant) against central
    differences of the real map, relative step 1e-4 (no branch changes; the
    differences' own error is at most 2.5e-6 here), for every output field."""
    from tests.helpers import rel_err, step_directions
    st, p, nxt = one_step
    assert st.epsbar.max() > 0 and st.T.max() > st.T.min()
    if field in OG.STEP_FIELDS:
        d = step_directions(st, np.random.default_rng(1))[field]
        jvp = OG.step_jvp(st, p, nxt, direction={field: d})
        e = 1e-4

        def G(sgn):
            s = st.copy()
            setattr(s, field, getattr(s, field) + sgn * e * d)
            return OG.step_map(s, p, nxt)
    else:
        jvp = OG.step_jvp(st, p, nxt, param=field)
        e = 1e-4 * abs(p[field])

        def G(sgn):
            return OG.step_map(st, dict(p, **{field: p[field] + sgn * e}), nxt)
    a, b = G(1), G(-1)
    errs = {o: rel_err(jvp[o], (getattr(a, o) - getattr(b, o)) / (2 * e)) for o in OG.STEP_FIELDS}
    bad = {o: v for o, v in errs.items() if not v < 2e-5}
    assert not bad, bad
