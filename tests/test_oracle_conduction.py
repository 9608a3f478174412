"""Pins of the oracle's heat conduction through the LME gradients (the
reading in oracle/conduction.py; the paper's chip-formation model itself is
adiabatic, Sec. 4.2).

* A uniform temperature stays uniform (partition of unity, sum grad N = 0).
* Conduction alone conserves the total heat sum m_p C_p T_p (insulated body).
* The MP gradient of an exactly linear nodal field is its slope (linear
  completeness of the LME gradients).
* On a bar at rest the two slowest cosine modes of the insulated heat
  equation decay at kappa / (rho C_p) (pi k / L)^2 within 5 %, so a lost
  factor (v_p, C_p, the mass weights), a sign error (growth) or a wrong
  operator (rate not scaling with k^2) fails.
"""
import numpy as np
import pytest

import otm_workloads as W
from oracle import conduction, step as OST


def _bar_state(T_of_x, **kw):
    w = W.heat_bar(**kw)
    p = W.params_from_workload(w)
    st = OST.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    st.T = T_of_x(st.xp)
    OST.assemble(st, p)            # h and Q of the prescribed field (q = 0)
    return w, p, st


def test_uniform_temperature_stays_uniform():
    w, p, st = _bar_state(lambda x: np.full(x.shape[0], 500.0), n=(9, 3, 3))
    for _ in range(50):
        OST.step(st, p)
    assert np.abs(st.T - 500.0).max() <= 1e-11 * 500.0
    assert np.abs(st.x - w.x_nodes).max() == 0.0      # nothing moves
    assert np.abs(st.q).max() <= 1e-9


def test_conduction_conserves_heat():
    rng = np.random.default_rng(0)
    w, p, st = _bar_state(lambda x: 300.0 + 50.0 * rng.random(x.shape[0]), n=(9, 4, 3))
    H0 = (st.mass * p["Cp"] * st.T).sum()
    OST.step(st, p)
    spread0 = st.T_nodes.std()
    for _ in range(100):
        OST.step(st, p)
    H1 = (st.mass * p["Cp"] * st.T).sum()
    assert abs(H1 - H0) <= 1e-13 * H0
    # and it smooths the field the nodes resolve (variation between the MPs
    # of one node's neighbourhood is not seen by the nodal projection)
    assert st.T_nodes.std() < 0.5 * spread0


def test_gradient_of_a_linear_nodal_field_is_its_slope():
    w, p, st = _bar_state(lambda x: np.zeros(x.shape[0]), n=(7, 5, 4))
    g = np.array([0.3, -1.7, 2.2])
    T_nodes = 4.0 + st.x @ g
    grad, dT = conduction.mp_terms(st.offsets, st.idx, st.N, st.dN, T_nodes,
                                   np.full(st.x.shape[0], 2.5), 0.1, OST._segsum)
    assert np.abs(grad - g).max() <= 1e-11 * np.abs(g).max()
    # a uniform nodal rate gives every MP dt * rate (partition of unity)
    assert np.abs(dT - 0.25).max() <= 1e-14


@pytest.mark.parametrize("k", [1, 2])
def test_cosine_mode_decays_at_the_diffusion_rate(k):
    L = 20.0
    steps = 400 if k == 1 else 150
    w, p, st = _bar_state(lambda x: 1.0 + 0.1 * np.cos(np.pi * k * x[:, 0] / L),
                          n=(21, 3, 3), kappa=1.0, rho0=1.0, Cp=1.0, dt=0.02, steps=steps)

    def amplitude(s):
        c = np.cos(np.pi * k * s.xp[:, 0] / L)
        c = c - (s.mass * c).sum() / s.mass.sum()
        return (s.mass * c * s.T).sum() / (s.mass * c * c).sum()

    a0 = amplitude(st)
    for _ in range(steps):
        OST.step(st, p)
    a1 = amplitude(st)
    t = steps * p["dt"]
    rate = -np.log(a1 / a0) / t
    exact = p["kappa"] / (p["rho0"] * p["Cp"]) * (np.pi * k / L) ** 2
    assert 0 < a1 < a0
    assert abs(rate / exact - 1.0) < 0.05, (rate, exact)
