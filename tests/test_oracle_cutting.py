"""Pins of the oracle's chip-formation pieces (Sec. 4.2): the Johnson-Cook
fracture criterion with stress triaxiality, the rigid tool's normal gap, the
penalty contact with Coulomb friction, and a short cut of a small workpiece."""
import math

import numpy as np
import pytest

import otm_workloads as W
from oracle import contact as CT
from oracle import material as M
from oracle import step as S


def _p(**over):
    w = W.config_by_name("small_cut")
    return dict(W.params_from_workload(w), **over)


def test_cutting_slab_has_the_papers_size():
    w = W.config_by_name("cutting_slab")
    # the paper's chip model: 27,417 nodes and 107,975 MPs
    assert w.n_nodes == 27633 and w.n_mp == 108000
    assert w.dt == 1e-10 and w.tool["r"] == 2e-6 and w.tool["mu"] == 0.8
    assert w.x_nodes[:, 0].min() >= 0.0


def test_triaxiality_of_textbook_states():
    s = np.zeros((5, 3, 3))
    s[0, 0, 0] = 3.0                               # uniaxial tension: 1/3
    s[1, 0, 0] = s[1, 1, 1] = 2.0                  # equibiaxial tension: 2/3
    s[2, 0, 1] = s[2, 1, 0] = 1.0                  # pure shear: 0
    s[3, 0, 0] = -5.0                              # uniaxial compression: -1/3
    s[4] = 7.0 * np.eye(3)                         # hydrostatic: no deviator -> 0
    eta = M.triaxiality(s)
    assert np.allclose(eta, [1 / 3, 2 / 3, 0.0, -1 / 3, 0.0], rtol=0, atol=1e-15)


def test_fracture_strain_closed_form():
    p = _p(jc_d=np.array([0.05, 0.3, -0.48, 0.02, 3.6]))
    d1, d2, d3, d4, d5 = p["jc_d"]
    dt, Tr, Tm = p["dt"], p["T_r"], p["T_m"]
    # quasi-static (rate below the reference rate) at room temperature
    ef = M.jc_fracture_strain(p, np.array([1 / 3]), np.array([0.1 * dt]), dt, np.array([Tr]))
    assert abs(ef[0] - (d1 + d2 * math.exp(d3 / 3))) < 1e-15
    # rate 1e6 x the reference, half-way to melting, triaxiality 0
    ef = M.jc_fracture_strain(p, np.array([0.0]), np.array([1e6 * dt]), dt,
                              np.array([0.5 * (Tr + Tm)]))
    want = (d1 + d2) * (1 + d4 * math.log(1e6)) * (1 + 0.5 * d5)
    assert abs(ef[0] - want) < 1e-14 * want
    # below T_r the temperature term is 1, above T_m it saturates
    lo = M.jc_fracture_strain(p, np.array([0.0]), np.array([0.0]), dt, np.array([Tr - 50]))
    hi = M.jc_fracture_strain(p, np.array([0.0]), np.array([0.0]), dt, np.array([Tm + 50]))
    assert abs(lo[0] - (d1 + d2)) < 1e-15 and abs(hi[0] - (d1 + d2) * (1 + d5)) < 1e-14


def _brute_gap(P, p, t):
    """Distance to the core wedge from dense samples of its two faces, minus
    the tip radius; negative inside (both face tests)."""
    r = p["tool_r"]
    a = p["tool_clearance"]
    c = np.asarray(p["tool_c"]) + t * np.asarray(p["tool_v"])
    s = np.linspace(0.0, 40 * r, 400001)
    face1 = c[:2] + s[:, None] * np.array([0.0, 1.0])
    face2 = c[:2] + s[:, None] * np.array([math.cos(a), math.sin(a)])
    pts = np.concatenate([face1, face2])
    out = []
    for q in P:
        dmin = np.sqrt(((pts - q[:2]) ** 2).sum(axis=1)).min()
        d = q[:2] - c[:2]
        # inside the core: to the right of the rake face and above the flank
        inside = d[0] >= 0 and d[1] * math.cos(a) >= d[0] * math.sin(a)
        out.append((-dmin if inside else dmin) - r)
    return np.array(out)


def test_tool_gap_against_dense_sampling():
    p = _p()
    rng = np.random.default_rng(3)
    r = p["tool_r"]
    c = np.asarray(p["tool_c"])
    t = 2e-9
    cx = c + t * np.asarray(p["tool_v"])
    P = np.zeros((300, 3))
    P[:, :2] = cx[:2] + rng.uniform(-6 * r, 6 * r, (300, 2))
    P[:, 2] = rng.uniform(0, 4e-6, 300)
    g, n = CT.tool_gap(P, t, p)
    want = _brute_gap(P, p, t)
    assert np.abs(g - want).max() < 1e-4 * r      # sample spacing 1e-4 r
    assert np.allclose((n * n).sum(axis=1), 1.0) and np.all(n[:, 2] == 0.0)
    # moving along the normal by the gap lands on the tool surface
    g2, _ = CT.tool_gap(P - g[:, None] * n, t, p)
    assert np.abs(g2).max() < 1e-12 * r


def test_normal_penalty_and_no_friction_for_normal_motion():
    """A node at rest 3 nm inside the rake face (above the tip) while the tool
    moves along the face normal: force c_N * 3 nm along -x, no friction."""
    p = _p()
    c = np.asarray(p["tool_c"])
    x = np.array([[c[0] - p["tool_r"] + 3e-9, c[1] + 5e-6, 1e-6]])
    f, gT = CT.tool_forces(x, np.zeros((1, 3)), np.zeros((1, 3)), 0.0, p)
    assert np.allclose(f, [[-p["tool_cN"] * 3e-9, 0, 0]], rtol=1e-9, atol=0)
    assert np.all(gT == 0)


@pytest.mark.parametrize("slide", [1e-12, 1e-8])
def test_stick_and_slip_on_the_flank(slide):
    """A node 2 nm inside the flank face slides along it (relative to the tool)
    by ``slide`` in one step: the tangential force is -c_T * slide while that
    is within mu times the normal force (stick), and mu times the normal force
    against the sliding direction once it is not (slip)."""
    p = _p()
    a = p["tool_clearance"]
    u2 = np.array([math.cos(a), math.sin(a), 0.0])
    n2 = np.array([math.sin(a), -math.cos(a), 0.0])
    c = np.asarray(p["tool_c"])
    x = (c + 5 * p["tool_r"] * u2 + (p["tool_r"] - 2e-9) * n2)[None, :]
    du = (p["dt"] * np.asarray(p["tool_v"]) + slide * u2)[None, :]
    f, gT = CT.tool_forces(x, du, np.zeros((1, 3)), 0.0, p)
    fn = p["tool_cN"] * 2e-9
    ft = f[0] - (f[0] @ n2) * n2
    assert abs(f[0] @ n2 - fn) < 1e-9 * fn
    if p["tool_cT"] * slide <= p["tool_mu"] * fn:
        assert np.allclose(ft, -p["tool_cT"] * slide * u2, rtol=1e-6, atol=1e-12 * fn)
        assert np.allclose(gT[0], slide * u2, rtol=1e-6, atol=1e-20)
    else:
        assert np.allclose(ft, -p["tool_mu"] * fn * u2, rtol=1e-9, atol=1e-12 * fn)
        assert np.allclose(gT[0], p["tool_mu"] * fn / p["tool_cT"] * u2, rtol=1e-9)


@pytest.fixture(scope="module")
def cut_run():
    w = W.config_by_name("small_cut")
    p = W.params_from_workload(w)
    st = S.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    hist = []
    for _ in range(w.steps):
        prev = st.copy()
        S.step(st, p)
        hist.append((prev, st.copy()))
    return w, p, hist


def test_short_cut_contact_friction_and_fracture(cut_run):
    w, p, hist = cut_run
    last = hist[-1][1]
    assert last.failed.sum() > 10 and (last.epsbar > 0).sum() > 50
    g, n = CT.tool_gap(last.x, last.clock, p)
    assert (g < 0).sum() > 5 and -g.min() < 0.05 * w.h   # penalty keeps penetration small
    for prev, st in hist:
        # failure is irreversible; failed MPs carry no stress and keep their
        # plastic strain and temperature
        assert np.all(st.failed[prev.failed])
        assert np.all(st.sigma[st.failed] == 0.0)
        keep = prev.failed
        assert np.array_equal(st.epsbar[keep], prev.epsbar[keep])
        assert np.array_equal(st.T[keep], prev.T[keep])
        # an MP fails only once it has flowed
        assert np.all(st.epsbar[st.failed & ~prev.failed] > 0)
        # mass is conserved by the lumping, failed MPs included
        assert abs(st.m.sum() - w.mass_mp.sum()) < 1e-12 * w.mass_mp.sum()
        # nodes out of contact carry no tangential gap; Coulomb bound holds
        gp, npr = CT.tool_gap(prev.x, prev.clock, p)
        assert np.all(st.gT[gp >= 0] == 0.0)
        tT = -p["tool_cT"] * st.gT
        tn = p["tool_cN"] * np.maximum(-gp, 0.0)
        assert np.all(np.sqrt((tT * tT).sum(1)) <= p["tool_mu"] * tn * (1 + 1e-12))
    assert abs(last.clock - w.steps * w.dt) < 1e-12 * w.steps * w.dt


def test_light_node_penalty_is_limited_by_its_mass():
    """The node 3 nm inside the rake face: with a lumped mass m below
    c_N dt^2 the normal force is (m / dt^2) 3 nm; with a heavier node it is
    c_N 3 nm; a node without mass feels none."""
    p = _p()
    c = np.asarray(p["tool_c"])
    x = np.array([[c[0] - p["tool_r"] + 3e-9, c[1] + 5e-6, 1e-6]] * 3)
    k = p["tool_cN"] * p["dt"] ** 2
    m = np.array([0.1 * k, 10.0 * k, 0.0])
    f, gT = CT.tool_forces(x, np.zeros((3, 3)), np.zeros((3, 3)), 0.0, p, m)
    assert np.allclose(f[0], [-0.1 * p["tool_cN"] * 3e-9, 0, 0], rtol=1e-9, atol=0)
    assert np.allclose(f[1], [-p["tool_cN"] * 3e-9, 0, 0], rtol=1e-9, atol=0)
    assert np.all(f[2] == 0) and np.all(gT == 0)


@pytest.mark.parametrize("limited", [True, False])
def test_limited_penalty_keeps_a_light_node_bounded(limited):
    """One light node (m = 0.01 c_N dt^2) released 3 nm inside a resting tool,
    moved by the central difference with the contact force alone: with the
    mass limit one step puts it back on the surface and it leaves at 3 nm per
    step, its penetration never exceeding the initial 3 nm; without the limit
    the contact spring's frequency is beyond 2 / dt and one step fires it off
    at 100 times that (c_N dt^2 / m = 100)."""
    p = _p(tool_v=np.zeros(3))
    c = np.asarray(p["tool_c"])
    dt2 = p["dt"] ** 2
    m = np.array([0.01 * p["tool_cN"] * dt2])
    x = np.array([[c[0] - p["tool_r"] + 3e-9, c[1] + 5e-6, 1e-6]])
    du = np.zeros((1, 3))
    gT = np.zeros((1, 3))
    worst, fastest = 0.0, 0.0
    for _ in range(50):
        f, gT = CT.tool_forces(x, du, gT, 0.0, p, m if limited else None)
        du = du + dt2 * f / m[:, None]
        x = x + du
        g, _ = CT.tool_gap(x, 0.0, p)
        worst = max(worst, -g[0])
        fastest = max(fastest, float(np.sqrt((du * du).sum())))
    if limited:
        assert worst <= 3e-9 * (1 + 1e-9) and fastest <= 3e-9 * (1 + 1e-9)
    else:
        assert fastest >= 0.99 * 100 * 3e-9
