"""Pins of the oracle's Johnson-Cook fracture decision (Sec. 4.2 fracture
criterion: an MP fails once its equivalent plastic strain reaches the
critical strain at its stress triaxiality, plastic strain rate and
temperature).

Each case is one step of a coaxial stretch dF = diag(l1, l2, l2) from an
unstrained elastic state (b^e = 1) with a given hardening history (epsbar_n)
and temperature T_n.  For coaxial stretches the Hencky strains add, so the
step has a closed form that the test derives on its own (textbook radial
return with linear hardening):

  theta = ln l1 + 2 ln l2                  (volumetric strain, elastic)
  a_tr  = 2/3 |ln l1 - ln l2|              (equivalent deviatoric strain)
  q_tr  = 3 mu a_tr
  s     = 1 - T*_n^m                       (softening at T_n)
  depsbar = (q_tr - s (A + B epsbar_n)) / (3 mu + s B)   (JC with n = 1, C = 0)
  q     = q_tr - 3 mu depsbar,   epsbar_{n+1} = epsbar_n + depsbar
  T_{n+1} = T_n + chi q depsbar / (rho0 Cp)
  eta   = K theta / q                      (mean over von Mises stress; J cancels)

Every case puts epsbar_{n+1} strictly between the critical strain built from
the right ingredients and the one built from a plausible wrong ingredient, so
the oracle's decision tells them apart:

* epsbar_{n+1}, not epsbar_n and not the increment depsbar;
* T_{n+1} (after this step's heating), not T_n;
* eta of the returned stress, not of the trial stress;
* the rate depsbar / dt of this step;
* an MP that has never yielded does not fail, even for a critical strain <= 0.
"""
import types

import numpy as np
import pytest

from oracle import material as M
from oracle import step as OST

E, NU = 200e9, 0.3
MU = E / (2 * (1 + NU))
K = E / (3 * (1 - 2 * NU))


def params(**over):
    p = dict(model=M.J2_JC, E=E, nu=NU, rho0=8000.0, Cp=500.0, chi=0.9, A=300e6, B=500e6,
             n=1.0, C=0.0, m=1.0, eps_dot0=1.0, T_r=300.0, T_m=1300.0, dt=1e-6,
             jc_d=(0.1, 0.0, 0.0, 0.0, 0.0), fracture=True, rm_tol=1e-14, rm_max_iter=60)
    p.update(over)
    return p


def closed_form(p, l1, l2, eb_n, T_n):
    """(depsbar, epsbar_{n+1}, T_{n+1}, eta, eta_trial) of one coaxial step."""
    ln1, ln2 = np.log(l1), np.log(l2)
    theta = ln1 + 2.0 * ln2
    q_tr = 3.0 * MU * (2.0 / 3.0) * abs(ln1 - ln2)
    ts_n = min(max((T_n - p["T_r"]) / (p["T_m"] - p["T_r"]), 0.0), 1.0)
    s = 1.0 - ts_n ** p["m"]
    deps = max(0.0, (q_tr - s * (p["A"] + p["B"] * eb_n)) / (3.0 * MU + s * p["B"]))
    q = q_tr - 3.0 * MU * deps
    T1 = T_n + p["chi"] * q * deps / (p["rho0"] * p["Cp"])
    return deps, eb_n + deps, T1, K * theta / q, K * theta / q_tr


def crit(p, eta, deps, T):
    """Johnson-Cook critical strain from its printed factors (Sec. 4.2)."""
    d1, d2, d3, d4, d5 = p["jc_d"]
    rate = max(deps / (p["dt"] * p["eps_dot0"]), 1.0)
    ts = min(max((T - p["T_r"]) / (p["T_m"] - p["T_r"]), 0.0), 1.0)
    return (d1 + d2 * np.exp(d3 * eta)) * (1 + d4 * np.log(rate)) * (1 + d5 * ts)


def oracle_step(p, l1, l2, eb_n, T_n):
    """One step of the oracle's J2 update with the fracture check on MPs
    given as arrays (all alive, b^e = 1)."""
    l1, l2 = np.atleast_1d(l1).astype(float), np.atleast_1d(l2).astype(float)
    n = l1.size
    dF = np.zeros((n, 3, 3))
    dF[:, 0, 0], dF[:, 1, 1], dF[:, 2, 2] = l1, l2, l2
    st = types.SimpleNamespace(
        failed=np.zeros(n, bool), sigma=np.zeros((n, 3, 3)), be=np.tile(np.eye(3), (n, 1, 1)),
        epsbar=np.broadcast_to(np.asarray(eb_n, float), (n,)).copy(),
        T=np.broadcast_to(np.asarray(T_n, float), (n,)).copy())
    OST._update_with_fracture(st, p, dF, M.det3(dF))
    return st


def test_closed_form_matches_the_oracle_step():
    """The closed form above is the oracle's step (same epsbar, T, eta)."""
    p = params(jc_d=(10.0, 0.0, 0.0, 0.0, 0.0))
    l1, l2, eb_n, T_n = np.exp(0.02), np.exp(-0.009), 0.05, 450.0
    deps, eb1, T1, eta, _ = closed_form(p, l1, l2, eb_n, T_n)
    st = oracle_step(p, l1, l2, eb_n, T_n)
    assert not st.failed[0]
    assert abs(st.epsbar[0] - eb1) <= 1e-12 * eb1
    assert abs(st.T[0] - T1) <= 1e-12 * T1
    assert abs(M.triaxiality(st.sigma)[0] - eta) <= 1e-10 * abs(eta)
    assert deps > 0


def _case(p, l1, l2, eb_n, T_n):
    deps, eb1, T1, eta, eta_tr = closed_form(p, l1, l2, eb_n, T_n)
    return dict(deps=deps, eb1=eb1, T1=T1, eta=eta, eta_tr=eta_tr)


def test_decision_uses_the_new_equivalent_plastic_strain():
    """epsbar_n < eps_f <= epsbar_{n+1} and depsbar < eps_f: fails only when
    the strain after the step is compared."""
    l1, l2 = np.exp(0.02), np.exp(-0.01)
    p0 = params()
    c = _case(p0, l1, l2, 0.08, 300.0)
    d1 = c["eb1"] - 0.25 * c["deps"]             # between epsbar_n and epsbar_{n+1}
    p = params(jc_d=(d1, 0.0, 0.0, 0.0, 0.0))
    assert 0.08 < d1 <= c["eb1"] and c["deps"] < d1
    st = oracle_step(p, [l1, l1], [l2, l2], [0.08, 0.0], 300.0)
    # the second MP starts unhardened: epsbar_{n+1} = depsbar < eps_f
    assert st.failed.tolist() == [True, False]
    assert np.all(st.sigma[0] == 0.0) and np.abs(st.sigma[1]).max() > 0


def test_decision_uses_the_temperature_after_heating():
    """Strong heating (small rho0 Cp) moves T* from 0.1 to ~0.5 within the
    step; with d5 = 2 the critical strain at T_{n+1} exceeds epsbar_{n+1}
    while the one at T_n does not."""
    l1, l2 = np.exp(0.02), np.exp(-0.01)
    p0 = params(rho0=8000.0, Cp=1.5)
    c = _case(p0, l1, l2, 0.0, 400.0)
    ts_n = 0.1
    ts_1 = (c["T1"] - 300.0) / 1000.0
    assert 0.3 < ts_1 < 0.9
    # eps_f(T) = d1 (1 + 2 T*): put epsbar_{n+1} in the middle of the gap
    d1 = c["eb1"] / (1 + 2 * 0.5 * (ts_n + ts_1))
    p = params(rho0=8000.0, Cp=1.5, jc_d=(d1, 0.0, 0.0, 0.0, 2.0))
    assert crit(p, 0.0, 0.0, 400.0) < c["eb1"] < crit(p, 0.0, 0.0, c["T1"])
    st = oracle_step(p, l1, l2, 0.0, 400.0)
    assert not st.failed[0]
    assert abs(st.T[0] - c["T1"]) <= 1e-12 * c["T1"]
    # without the temperature factor the same step fails
    p_cold = params(rho0=8000.0, Cp=1.5, jc_d=(d1, 0.0, 0.0, 0.0, 0.0))
    assert oracle_step(p_cold, l1, l2, 0.0, 400.0).failed[0]


def test_decision_uses_the_triaxiality_of_the_returned_stress():
    """A volumetric part makes eta = K theta / q; the return lowers q far
    below q_tr, so eta is well above its trial value.  With d3 < 0 the
    critical strain at the returned eta lies below epsbar_{n+1} and the one
    at the trial eta above it."""
    l1, l2 = np.exp(0.02), np.exp(-0.008)         # theta = 0.004 > 0
    p0 = params()
    c = _case(p0, l1, l2, 0.0, 300.0)
    assert c["eta"] > 3 * c["eta_tr"] > 0
    # eps_f = d2 exp(-2 eta): epsbar_{n+1} at the geometric middle
    d2 = c["eb1"] * np.exp(2.0 * 0.5 * (c["eta"] + c["eta_tr"]))
    p = params(jc_d=(0.0, d2, -2.0, 0.0, 0.0))
    assert crit(p, c["eta"], 0.0, 300.0) < c["eb1"] < crit(p, c["eta_tr"], 0.0, 300.0)
    st = oracle_step(p, l1, l2, 0.0, 300.0)
    assert st.failed[0]
    # the same step in pure shear-free compression of volume (theta < 0):
    # eta < 0 raises eps_f above epsbar_{n+1}, no failure
    l2c = np.exp(-0.012)
    cc = _case(p, l1, l2c, 0.0, 300.0)
    assert cc["eta"] < 0 and crit(p, cc["eta"], 0.0, 300.0) > cc["eb1"]
    assert not oracle_step(p, l1, l2c, 0.0, 300.0).failed[0]


def test_decision_uses_this_steps_plastic_rate():
    """rate* = depsbar / (dt rate0) ~ 1.9e4 here; with d4 = 0.1 the rate
    factor is ~2, and epsbar_{n+1} sits between d1 and the rate-scaled
    critical strain.  With a reference rate above the step's rate the factor
    is 1 and the MP fails."""
    l1, l2 = np.exp(0.02), np.exp(-0.01)
    p0 = params()
    c = _case(p0, l1, l2, 0.0, 300.0)
    rate = c["deps"] / p0["dt"]
    assert rate > 1e3
    fac = 1 + 0.1 * np.log(rate)
    d1 = c["eb1"] / (0.5 * (1 + fac))
    p = params(jc_d=(d1, 0.0, 0.0, 0.1, 0.0))
    assert d1 < c["eb1"] < crit(p, 0.0, c["deps"], 300.0)
    assert not oracle_step(p, l1, l2, 0.0, 300.0).failed[0]
    p_slow = params(jc_d=(d1, 0.0, 0.0, 0.1, 0.0), eps_dot0=10 * rate)
    assert oracle_step(p_slow, l1, l2, 0.0, 300.0).failed[0]


def test_an_mp_that_never_yielded_does_not_fail():
    """d1 < 0 makes the critical strain negative: an elastic MP with
    epsbar = 0 still does not fail, an elastic MP hardened before fails, and
    so does a yielding one."""
    p = params(jc_d=(-0.05, 0.0, 0.0, 0.0, 0.0))
    small = np.exp(1e-5)                               # q_tr far below the yield stress
    big = np.exp(0.02)
    st = oracle_step(p, [small, small, big], [1.0, 1.0, np.exp(-0.01)], [0.0, 0.01, 0.0],
                     300.0)
    assert st.epsbar[0] == 0.0 and st.epsbar[1] == 0.01 and st.epsbar[2] > 0
    assert st.failed.tolist() == [False, True, True]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_coaxial_steps_follow_the_closed_form_decision(seed):
    """Random stretches, histories and constants: the oracle fails exactly
    the MPs whose closed-form epsbar_{n+1} reaches the closed-form critical
    strain (cases within 1e-9 of the threshold are skipped)."""
    rng = np.random.default_rng(seed)
    n = 200
    ln1 = rng.uniform(-0.01, 0.03, n)
    ln2 = rng.uniform(-0.015, 0.005, n)
    eb_n = rng.uniform(0.0, 0.2, n) * (rng.random(n) < 0.8)
    T_n = rng.uniform(300.0, 700.0, n)
    d = (rng.uniform(-0.05, 0.1), rng.uniform(0.05, 0.3), rng.uniform(-2.0, -0.5),
         rng.uniform(0.0, 0.05), rng.uniform(0.0, 2.0))
    p = params(jc_d=d, Cp=rng.uniform(5.0, 50.0))
    st = oracle_step(p, np.exp(ln1), np.exp(ln2), eb_n, T_n)
    want, keep = [], []
    for k in range(n):
        deps, eb1, T1, eta, _ = closed_form(p, np.exp(ln1[k]), np.exp(ln2[k]), eb_n[k], T_n[k])
        ef = crit(p, eta, deps, T1)
        keep.append(abs(eb1 - ef) > 1e-9 * max(1.0, abs(ef)))
        want.append(eb1 > 0 and eb1 >= ef)
    keep = np.array(keep)
    assert keep.sum() > 150
    assert np.array_equal(st.failed[keep], np.array(want)[keep])
    assert 0 < np.sum(want) < n
