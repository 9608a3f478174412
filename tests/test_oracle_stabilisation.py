"""Pins of the oracle's stabilisation term (Sec. 2.1: the stabilised nodal
residual r_I - eps sum_p N_Ip e_Ip and the under-integration error e_Ip).

e_Ip compares the pair's new relative position with its previous one mapped
by the MP's deformation-gradient increment, so it vanishes for every affine
motion of the nodes (the LME functions reproduce linear fields, so x_p and
dF follow the motion exactly), and for one non-affine motion of a symmetric
patch it has a closed form derived below from linear reproduction alone."""
import numpy as np
import pytest

from oracle import step as S
import otm_workloads as inputs


def _affine_step(w, p, G, shift):
    """One step in which every node moves by the affine map x -> G x + shift."""
    st = S.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    st.du = st.x @ (G - np.eye(3)).T + shift
    st.f[:] = 0.0
    S.node_update(st, p)
    S.mp_update(st, p)
    S.rebuild_lists(st, p)
    S.shape(st, p)
    return st


def _mp_of_pair(st):
    return np.repeat(np.arange(st.xp.shape[0]), np.diff(st.offsets))


@pytest.mark.parametrize("kind", ["stretch", "rotation", "translation"])
def test_error_vanishes_for_affine_motions(cube, kind):
    p = inputs.params_from_workload(cube)
    if kind == "stretch":
        G = np.eye(3) + 1e-3 * np.array([[1.0, 0.3, -0.2], [0.1, -0.5, 0.4], [0.25, 0.0, 0.7]])
    elif kind == "rotation":
        a = 0.3
        G = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1.0]])
    else:
        G = np.eye(3)
    st = _affine_step(cube, p, G, np.array([0.05, -0.02, 0.01]))
    e = S.underintegration_error(st, _mp_of_pair(st))
    # the LME consistency tolerance (1e-14 h) is the only source
    assert np.abs(e).max() < 1e-11
    # hence the stabilised force equals the unstabilised one to that level
    a, b = st.copy(), st.copy()
    S.assemble(a, dict(p, eps_stab=0.0))
    mu = cube.material.E / (2 * (1 + cube.material.nu))
    S.assemble(b, dict(p, eps_stab=mu * cube.h ** 2))
    assert np.abs(b.f - a.f).max() <= 1e-10 * mu * cube.h ** 2
    assert np.array_equal(a.m, b.m)


def _corner_patch(a=1.0):
    """Eight nodes at the corners (+-a, +-a, +-a) of a cube and one MP at its
    centre, every corner in the MP's support."""
    corners = np.array([[a if c & 1 else -a, a if c & 2 else -a, a if c & 4 else -a]
                        for c in range(8)], float)
    p = dict(model=inputs.MODEL_NEOHOOKE, E=1.0, nu=0.3, rho0=1.0, beta=0.5 / a ** 2,
             lme_tol=1e-15 * a, lme_max_iter=50, dt=1e-3, wall=False, wall_x=np.zeros(3),
             wall_n=np.array([0, 0, 1.0]), T_r=293.0, rebuild_every=1)
    lists = (np.array([0, 8], np.int64), np.arange(8, dtype=np.int32))
    st = S.init_state(corners, np.zeros((1, 3)), np.ones(1), np.ones(1), np.zeros((8, 3)), p,
                      lists=lists)
    return st, p, corners


def test_error_closed_form_for_a_moved_corner():
    """One corner J of the symmetric patch moves by delta, the others stay.
    By symmetry lambda = 0 and N_I = 1/8; linear reproduction then forces
    grad N_I = d_I / (8 a^2) with d_I = x_I - x_p.  Hence x_p' = x_p + delta/8,
    dF = 1 + delta (x) d_J / (8 a^2), and with |d_I| = sqrt(3) a
      e_I = delta ([I = J] - 1/8 - d_J . d_I / (8 a^2)) / (sqrt(3) a):
    delta / (2 sqrt 3 a) at J, delta / (4 sqrt 3 a) at the opposite corner,
    -delta / (4 sqrt 3 a) at the three corners sharing an edge with J and 0
    at the three sharing only a face."""
    a = 0.7
    st, p, X = _corner_patch(a)
    assert np.abs(st.N - 0.125).max() < 1e-15 and np.abs(st.lam).max() < 1e-12
    J = 5
    delta = np.array([0.013, -0.004, 0.021]) * a
    st.du = np.zeros((8, 3))
    st.du[J] = delta
    st.f[:] = 0.0
    S.node_update(st, p)
    S.mp_update(st, p)
    e = S.underintegration_error(st, np.zeros(8, dtype=np.int64))
    dJ = X[J]
    expect = np.empty((8, 3))
    for I in range(8):
        coef = (1.0 if I == J else 0.0) - 0.125 - dJ @ X[I] / (8 * a * a)
        expect[I] = delta * coef / (np.sqrt(3.0) * a)
    assert np.abs(e - expect).max() < 1e-13 * np.abs(delta).max() / a
    s3 = np.sqrt(3.0) * a
    shared = (X * dJ > 0).sum(axis=1)          # coordinates shared with corner J
    assert np.allclose(e[J], delta / (2 * s3), rtol=0, atol=1e-15)
    assert np.allclose(e[shared == 0], delta / (4 * s3), rtol=0, atol=1e-15)
    assert np.allclose(e[shared == 2], -delta / (4 * s3), rtol=0, atol=1e-15)
    assert np.allclose(e[shared == 1], 0.0, rtol=0, atol=1e-15)


def test_term_is_linear_in_eps_and_absent_at_t0(cube):
    """The stabilised force is f(0) - eps * s with s independent of eps, and
    the t = 0 assembly (no previous configuration) carries no term."""
    p = inputs.params_from_workload(cube)
    mu = cube.material.E / (2 * (1 + cube.material.nu))
    eps = mu * cube.h ** 2
    st0 = S.init_state(cube.x_nodes, cube.x_mp, cube.vol_mp, cube.mass_mp, cube.v0_nodes, p)
    st1 = S.init_state(cube.x_nodes, cube.x_mp, cube.vol_mp, cube.mass_mp, cube.v0_nodes,
                       dict(p, eps_stab=eps))
    assert np.array_equal(st0.f, st1.f)
    rng = np.random.default_rng(4)
    st0.du = st0.du + 1e-3 * cube.h * rng.standard_normal(st0.du.shape)   # non-affine
    S.node_update(st0, p)
    S.mp_update(st0, p)
    S.shape(st0, p)
    fs = []
    for k in (0.0, 1.0, 2.5):
        s = st0.copy()
        S.assemble(s, dict(p, eps_stab=k * eps))
        fs.append(s.f)
    d1, d2 = fs[1] - fs[0], fs[2] - fs[0]
    assert np.abs(d1).max() > 1e-6 * np.abs(fs[0]).max()      # the term is felt
    assert np.abs(d2 - 2.5 * d1).max() < 1e-9 * np.abs(d2).max()
