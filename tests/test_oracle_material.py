"""Pins of the oracle's constitutive updates (Sec. 4.1, Sec. 4.2)."""
import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

from oracle import material as M

E, NU = 117e9, 0.35
LAM, MU = M.lame(E, NU)
KB = LAM + 2 * MU / 3


def jc(**over):
    p = dict(model=M.J2_JC, E=E, nu=NU, rho0=8930.0, A=90e6, B=292e6, n=0.31, C=0.025,
             m=1.09, eps_dot0=1.0, T_r=293.0, T_m=1356.0, Cp=385.0, chi=0.9, Y0=0, H=0)
    p.update(over)
    return p


def rand_spd(rng, n, scale):
    A = np.eye(3) + scale * rng.standard_normal((n, 3, 3))
    return A @ np.swapaxes(A, 1, 2)


def rand_dF(rng, n, scale):
    return np.eye(3) + scale * rng.standard_normal((n, 3, 3))


def test_sym_log_exp_against_scipy():
    rng = np.random.default_rng(0)
    B = rand_spd(rng, 8, 0.03)     # within the series' range |b - 1| < 0.5
    for b in B:
        assert np.abs(M.sym_log_eigh(b[None])[0] - scipy.linalg.logm(b).real).max() < 1e-13
        assert np.abs(M.sym_log_series(b[None])[0] - scipy.linalg.logm(b).real).max() < 1e-13
        a = 0.5 * (b + b.T) - np.eye(3)
        assert np.abs(M.sym_exp_eigh(a[None])[0] - scipy.linalg.expm(a)).max() < 1e-13
        assert np.abs(M.sym_exp_series(a[None])[0] - scipy.linalg.expm(a)).max() < 1e-13


def test_neo_hooke_small_strain_is_linear_elasticity():
    rng = np.random.default_rng(1)
    G = rng.standard_normal((3, 3))
    errs = []
    for t in (1e-3, 1e-4):
        F = np.eye(3) + t * G
        eps = 0.5 * t * (G + G.T)
        lin = LAM * np.trace(eps) * np.eye(3) + 2 * MU * eps
        errs.append(np.abs(M.neo_hooke_cauchy(F[None], E, NU)[0] - lin).max() / (E * t))
    # the remainder is second order in the strain: relative to E t it
    # drops 10x for a 10x smaller strain
    assert 8 < errs[0] / errs[1] < 12 and errs[1] < 1e-3


def test_neo_hooke_rotation_and_zero():
    th = 0.3
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    assert np.abs(M.neo_hooke_cauchy(R[None], E, NU)).max() < 1e-15 * E
    U = np.diag([1.01, 0.99, 1.002])
    s1 = M.neo_hooke_cauchy(U[None], E, NU)[0]
    s2 = M.neo_hooke_cauchy((R @ U)[None], E, NU)[0]
    assert np.abs(R @ s1 @ R.T - s2).max() < 1e-6 * E * 1e-6


def _upd(p, dF, be=None, eb=None, T=None, dt=3e-9):
    n = dF.shape[0]
    be = np.tile(np.eye(3), (n, 1, 1)) if be is None else be
    eb = np.zeros(n) if eb is None else eb
    T = np.full(n, p["T_r"]) if T is None else T
    J = M.det3(dF)
    return M.j2_update(p, dF, be, eb, T, J, dt)


def test_j2_small_strain_elastic_is_linear_elasticity():
    p = jc()
    rng = np.random.default_rng(2)
    G = rng.standard_normal((3, 3))
    errs = []
    for t in (1e-4, 1e-5):           # q_tr well below A: elastic
        dF = (np.eye(3) + t * G)[None]
        sig, be, eb, T, de = _upd(p, dF)
        assert de[0] == 0 and eb[0] == 0
        eps = 0.5 * t * (G + G.T)
        lin = LAM * np.trace(eps) * np.eye(3) + 2 * MU * eps
        errs.append(np.abs(sig[0] - lin).max() / (E * t))
    assert 8 < errs[0] / errs[1] < 12 and errs[1] < 1e-3


def test_j2_volumetric_closed_form():
    """Pure dilatation has no deviator: sigma = K ln(J) / J 1 (Hencky)."""
    p = jc()
    for a in (0.97, 1.0, 1.02):
        sig, be, eb, T, de = _upd(p, (a * np.eye(3))[None])
        J = a ** 3
        assert np.abs(sig[0] - KB * np.log(J) / J * np.eye(3)).max() < 1e-12 * KB
        assert np.abs(be[0] - a * a * np.eye(3)).max() < 1e-14


def test_j2_plastic_consistency_and_volume_preservation():
    p = jc()
    rng = np.random.default_rng(3)
    dF = rand_dF(rng, 64, 0.01)
    be0 = rand_spd(rng, 64, 0.001)
    eb0 = rng.uniform(0, 0.2, 64)
    T0 = rng.uniform(293, 700, 64)
    dt = 3e-9
    J = M.det3(dF)
    sig, be, eb, T, de = M.j2_update(p, dF, be0, eb0, T0, J, dt)
    btr = dF @ be0 @ np.swapaxes(dF, 1, 2)
    assert np.all(de >= 0) and (de > 0).sum() > 32
    pl = de > 0
    # consistency: q_{n+1} = sigma_Y(epsbar_{n+1}, deps/dt, T_n) on the plastic MPs
    tau = sig * J[:, None, None]
    s = tau - np.trace(tau, axis1=1, axis2=2)[:, None, None] / 3 * np.eye(3)
    q = np.sqrt(1.5 * (s * s).sum(axis=(1, 2)))
    sy, _ = M.flow_stress(p, eb0, de, dt, M.homologous_T(p, T0))
    assert np.abs(q[pl] - sy[pl]).max() < 1e-9 * sy.max()
    # elastic MPs stay inside the yield surface
    sy0, _ = M.flow_stress(p, eb0, 0 * de, dt, M.homologous_T(p, T0))
    assert np.all(q[~pl] <= sy0[~pl] * (1 + 1e-12))
    # the exponential map keeps det b^e (plastic flow is isochoric)
    assert np.abs(M.det3(be) / M.det3(btr) - 1).max() < 1e-13
    # heating closed form
    dT = p["chi"] * q * de / (p["rho0"] * p["Cp"])
    assert np.abs(T - T0 - dT).max() < 1e-12 * T0.max()
    assert np.array_equal(eb, eb0 + de)
    # return is radial: dev log b^e_new is parallel to dev log b^e_tr
    lnb = M.sym_log_eigh(be)
    lnt = M.sym_log_eigh(btr)
    dv = lambda A: A - np.trace(A, axis1=1, axis2=2)[:, None, None] / 3 * np.eye(3)
    a, b = dv(lnb)[pl].reshape(-1, 9), dv(lnt)[pl].reshape(-1, 9)
    cos = (a * b).sum(1) / np.linalg.norm(a, axis=1) / np.linalg.norm(b, axis=1)
    assert np.abs(cos - 1).max() < 1e-10


def test_return_root_matches_brentq():
    p = jc()
    rng = np.random.default_rng(4)
    q = rng.uniform(150e6, 900e6, 40)
    eb = rng.uniform(0, 0.5, 40)
    eb[:5] = 0.0
    Ts = rng.uniform(0, 0.6, 40)
    dt = 3e-9
    x, _ = M.solve_return(p, q, eb, Ts, dt, MU)
    for k in range(40):
        g = lambda y: q[k] - 3 * MU * y - M.flow_stress(p, eb[k:k + 1], np.array([y]), dt,
                                                         Ts[k:k + 1])[0][0]
        if g(0.0) <= 0:
            continue
        ref = scipy.optimize.brentq(g, 0.0, q[k] / (3 * MU), xtol=1e-300, rtol=8.9e-16)
        # the root is fixed only up to the rounding of g (~eps q_tr) over its
        # slope (>= 3 mu)
        assert abs(x[k] - ref) <= 8 * 2.2e-16 * q[k] / (3 * MU) + 4e-15 * ref


def test_linear_hardening_closed_form():
    """J2_LINEAR and JC with C = 0, T = T_r, n = 1, B = H both give the
    textbook radial return deps = (q_tr - sigma_Y0) / (3 mu + H)."""
    H, Y0 = 100e6, 400e6
    rng = np.random.default_rng(5)
    dF = rand_dF(rng, 32, 0.02)
    eb0 = rng.uniform(0, 0.1, 32)
    for p in (dict(jc(model=M.J2_LINEAR, Y0=Y0, H=H)), jc(A=Y0, B=H, n=1.0, C=0.0)):
        J = M.det3(dF)
        be0 = np.tile(np.eye(3), (32, 1, 1))
        sig, be, eb, T, de = M.j2_update(p, dF, be0, eb0, np.full(32, 293.0), J, 3e-9)
        lnb = 0.5 * M.sym_log_eigh(dF @ np.swapaxes(dF, 1, 2))
        dv = lnb - np.trace(lnb, axis1=1, axis2=2)[:, None, None] / 3 * np.eye(3)
        qtr = np.sqrt(1.5 * ((2 * MU * dv) ** 2).sum(axis=(1, 2)))
        expect = np.maximum(qtr - (Y0 + H * eb0), 0) / (3 * MU + H)
        assert (expect > 0).sum() > 10
        assert np.abs(de - expect).max() < 1e-13 * expect.max()
        if p["model"] == M.J2_LINEAR:
            assert np.array_equal(T, np.full(32, 293.0))


def test_thermal_softening_clamp():
    p = jc()
    Ts = M.homologous_T(p, np.array([100.0, 293.0, 800.0, 2000.0]))
    assert np.array_equal(Ts, [0.0, 0.0, (800 - 293) / (1356 - 293), 1.0])
    sy, _ = M.flow_stress(p, np.array([0.1] * 4), np.zeros(4), 1e-9, Ts)
    assert sy[3] == 0.0 and sy[0] == sy[1] and sy[2] < sy[1]


def test_complex_step_variant_matches_real():
    """The holomorphic (series) variant used for complex-step derivatives
    reproduces the eigen-decomposition oracle."""
    p = jc()
    rng = np.random.default_rng(6)
    dF = rand_dF(rng, 16, 0.01)
    be0 = rand_spd(rng, 16, 0.001)
    eb0 = rng.uniform(0, 0.2, 16)
    T0 = rng.uniform(293, 500, 16)
    J = M.det3(dF)
    a = M.j2_update(p, dF, be0, eb0, T0, J, 3e-9)
    b = M.j2_update(p, dF.astype(complex), be0.astype(complex), eb0.astype(complex),
                    T0.astype(complex), J.astype(complex), 3e-9, spectral="series", polish=2)
    for u, v in zip(a, b):
        assert np.abs(u - v.real).max() <= 1e-13 * max(1.0, np.abs(u).max())
    # derivative w.r.t. A: complex step vs central difference
    hA = 1e-20 * p["A"]
    pc = dict(p, A=p["A"] + 1j * hA)
    c = M.j2_update(pc, dF.astype(complex), be0.astype(complex), eb0.astype(complex),
                    T0.astype(complex), J.astype(complex), 3e-9, spectral="series", polish=2)
    dsig_cs = c[0].imag / hA
    e = 1e-6 * p["A"]
    sp = M.j2_update(dict(p, A=p["A"] + e), dF, be0, eb0, T0, J, 3e-9)[0]
    sm = M.j2_update(dict(p, A=p["A"] - e), dF, be0, eb0, T0, J, 3e-9)[0]
    fd = (sp - sm) / (2 * e)
    assert np.abs(dsig_cs - fd).max() < 1e-6 * np.abs(fd).max()


def test_flow_stress_worked_example():
    """Johnson-Cook law (Sec. 4.2) on numbers chosen so that every factor is
    exact: A = 1, B = 1, n = 1/2 at epsbar = 0.25 gives 1.5; C = 0.1 at a
    rate ratio of e^2 gives 1.2; m = 1 at T* = 0.5 gives 0.5; product 0.9."""
    p = dict(model=M.J2_JC, A=1.0, B=1.0, n=0.5, C=0.1, m=1.0, eps_dot0=1.0,
             T_r=0.0, T_m=2.0)
    dt = 1.0
    de = np.array([np.exp(2.0)])
    eb = np.array([0.25]) - de
    sy, dsy = M.flow_stress(p, eb, de, dt, M.homologous_T(p, np.array([1.0])))
    assert abs(sy[0] - 0.9) < 1e-15
    # slope: d/dx [(1 + sqrt(e)) (1 + 0.1 ln x)] 0.5 at e = 0.25, x = e^2
    #   = (0.5 / sqrt(0.25) * 1.2 + 1.5 * 0.1 / e^2) * 0.5
    assert abs(dsy[0] - (1.0 * 1.2 + 1.5 * 0.1 / np.exp(2.0)) * 0.5) < 1e-15
    # below the reference rate the rate factor is 1
    sy2, _ = M.flow_stress(p, np.array([0.25 - 0.5]), np.array([0.5]), dt, np.array([0.5]))
    assert abs(sy2[0] - 0.75) < 1e-15
