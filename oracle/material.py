"""Constitutive updates at the material points (Alg. 1, step 4).

* Neo-Hookean (elastic cube workload; the paper names no elastic law for it):
  compressible form sigma = (mu / J)(b - 1) + (lambda ln J / J) 1, b = F F^T.
* Finite-strain J2 plasticity (Sec. 4.1): multiplicative split F = F^e F^p,
  Hencky strain eps^e = ln sqrt(b^e), exponential-map integration of the
  Lie-derivative flow rule, Kirchhoff stress tau = K tr(eps^e) 1 + 2 mu
  dev(eps^e), Cauchy stress sigma = tau / J.
* Flow stress: linear isotropic hardening sigma_Y = Y0 + H epsbar (Sec. 4.1
  yield function) or Johnson-Cook (Sec. 4.2 hardening law) with adiabatic
  heating dT = chi q dEpsbar / (rho0 C_p) (Sec. 4.2 temperature evolution).

Readings adopted where the printed formulas are garbled or silent:

* the exponential map is eps^e = eps^e,tr - dEpsbar (3/2) s^tr / q^tr (the
  printed 1/dt factor is dropped: the increment, not a rate, appears);
* the yield function is written with the von Mises form q - sigma_Y and the
  equivalent plastic strain increment dEpsbar (the Sec. 4.1 form in
  Delta-gamma is the same function scaled by sqrt(3/2));
* sigma = J^{-1} Q [K tr eps 1 + 2 mu dev eps] Q^T (the printed back
  transformation misses the 1/3 of the deviator and puts J on the wrong side);
* JC: plastic rate dEpsbar / dt, rate factor 1 + C ln(max(rate/rate0, 1)),
  homologous temperature clamped to [0, 1], softening evaluated at T_n and
  heating applied after the return (explicit stagger), heating uses the
  converged Kirchhoff equivalent stress with rho0 (tau_v / rho0 equals
  sigma_v / rho);
* the scalar return equation is solved by Newton safeguarded by bisection on
  [0, (q_tr - sigma_Y0) / (3 mu)], stopping when its residual is below 1e-14
  q_tr or the step or the bracket is below 1e-14 of the iterate.
"""
from __future__ import annotations

import numpy as np

NEOHOOKE, J2_JC, J2_LINEAR = 0, 1, 2


class ReturnMapNotConverged(RuntimeError):
    def __init__(self, mp_index):
        super().__init__(f"return map did not converge at material point {mp_index}")
        self.mp_index = mp_index


def lame(E, nu):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return lam, mu


def det3(A):
    return (A[..., 0, 0] * (A[..., 1, 1] * A[..., 2, 2] - A[..., 1, 2] * A[..., 2, 1])
            - A[..., 0, 1] * (A[..., 1, 0] * A[..., 2, 2] - A[..., 1, 2] * A[..., 2, 0])
            + A[..., 0, 2] * (A[..., 1, 0] * A[..., 2, 1] - A[..., 1, 1] * A[..., 2, 0]))


def neo_hooke_cauchy(F, E, nu):
    """sigma = (mu/J)(F F^T - 1) + (lambda ln J / J) 1."""
    lam, mu = lame(E, nu)
    J = det3(F)
    b = F @ np.swapaxes(F, -1, -2)
    I = np.eye(3)
    return (mu / J)[..., None, None] * (b - I) + (lam * np.log(J) / J)[..., None, None] * I


# ---------------------------------------------------------------- tensor log/exp
def sym_log_eigh(b):
    """Matrix logarithm of SPD matrices by the spectral theorem (float64)."""
    e, Q = np.linalg.eigh(b)
    return (Q * np.log(e)[..., None, :]) @ np.swapaxes(Q, -1, -2)


def sym_exp_eigh(a):
    e, Q = np.linalg.eigh(a)
    return (Q * np.exp(e)[..., None, :]) @ np.swapaxes(Q, -1, -2)


def _series_terms(D):
    nrm = np.sqrt((np.abs(D) ** 2).sum(axis=(-1, -2))).max() if D.size else 0.0
    if nrm >= 0.5:
        raise ValueError("series log/exp used outside its range")
    n = 4
    while nrm ** n / n > 1e-18 and n < 200:
        n += 1
    return n + 2


def sym_log_series(b):
    """log(1 + D) = sum_k (-1)^{k+1} D^k / k, holomorphic in the entries of b
    (used for complex-step derivatives)."""
    D = b - np.eye(3)
    nt = _series_terms(D)
    out = np.zeros_like(D)
    P = np.broadcast_to(np.eye(3), D.shape).astype(D.dtype)
    for k in range(1, nt + 1):
        P = P @ D
        out = out + ((-1) ** (k + 1) / k) * P
    return out


def sym_exp_series(a):
    """exp(a) = sum_k a^k / k! with scaling and squaring (holomorphic)."""
    nrm = np.sqrt((np.abs(a) ** 2).sum(axis=(-1, -2))).max() if a.size else 0.0
    s = max(0, int(np.ceil(np.log2(max(nrm, 1e-300) / 0.25)))) if nrm > 0.25 else 0
    A = a / 2.0 ** s
    out = np.broadcast_to(np.eye(3), a.shape).astype(a.dtype)
    term = out.copy()
    for k in range(1, 30):
        term = term @ A / k
        out = out + term
    for _ in range(s):
        out = out @ out
    return out


# ---------------------------------------------------------------- flow stress
def flow_stress(p, epsbar, deps, dt, Tstar):
    """sigma_Y and d sigma_Y / d deps at epsbar + deps, rate deps/dt."""
    if p["model"] == J2_LINEAR:
        return p["Y0"] + p["H"] * (epsbar + deps), p["H"] + 0 * deps
    A, B, n, C, m = p["A"], p["B"], p["n"], p["C"], p["m"]
    e = epsbar + deps
    pos = e.real > 0
    e_pos = np.where(pos, e, 1.0)
    hard = A + B * np.where(pos, e_pos ** n, 0.0)
    dhard = np.where(pos, B * n * e_pos ** (n - 1), 0.0)
    ratio = deps / (dt * p["eps_dot0"])
    above = ratio.real > 1.0
    ratio_safe = np.where(above, ratio, 1.0)
    rate = 1.0 + C * np.log(ratio_safe)
    deps_safe = np.where(above, deps, 1.0)
    drate = np.where(above, C / deps_safe, 0.0)
    Ts = np.where(Tstar.real > 0, Tstar, 1.0)
    therm = 1.0 - np.where(Tstar.real > 0, Ts ** m, 0.0)
    sy = hard * rate * therm
    # at epsbar + deps = 0 the slope is infinite for n < 1; callers ask for it
    # there only to discard it, and it is set to inf without forming inf * 0
    dsy = np.where(pos, (dhard * rate + hard * drate) * therm, np.inf)
    return sy, dsy


def homologous_T(p, T):
    if p["model"] != J2_JC:
        return np.zeros_like(T)
    ts = (T - p["T_r"]) / (p["T_m"] - p["T_r"])
    return np.where(ts.real < 0, 0.0 * ts, np.where(ts.real > 1, 1.0 + 0.0 * ts, ts))


def solve_return(p, q_tr, epsbar, Tstar, dt, mu, tol=1e-14, max_iter=60, polish=0):
    """Root of g(x) = q_tr - 3 mu x - sigma_Y(epsbar + x, x/dt, T*) on
    (0, x0], x0 = (q_tr - sigma_Y(epsbar, 0, T*)) / (3 mu), for MPs that
    yield; g is strictly decreasing so the root is unique.

    Newton from x0, bracket kept on the sign of g, bisection when the Newton
    iterate leaves the bracket.  Stops when the residual is at the rounding
    level, |g| <= tol q_tr (the only test that can end the iteration for MPs
    that barely yield, where the root is tiny), or when the Newton step or
    the bracket is below tol of the iterate.  ``polish`` extra Newton steps
    after convergence (complex-step runs)."""
    sy0, _ = flow_stress(p, epsbar, 0.0 * q_tr, dt, Tstar)
    x = (q_tr - sy0) / (3 * mu)
    lo = np.zeros_like(x.real)
    hi = x.real.copy()
    done = np.zeros(x.shape, dtype=bool)
    left = np.full(x.shape, polish)
    for _ in range(max_iter + polish):
        sy, dsy = flow_stress(p, epsbar, x, dt, Tstar)
        g = q_tr - 3 * mu * x - sy
        gp = -3 * mu - dsy
        polishing = done & (left > 0)
        left = np.where(polishing, left - 1, left)
        resid_ok = ~done & (np.abs(g.real) <= tol * q_tr.real)
        done = done | resid_ok
        active = ~done
        lo = np.where(active & (g.real > 0), x.real, lo)
        hi = np.where(active & (g.real <= 0), x.real, hi)
        xn = x - g / gp
        outside = ~((xn.real > lo) & (xn.real < hi)) & active
        xn = np.where(outside, 0.5 * (lo + hi), xn)
        small = (np.abs(xn.real - x.real) <= tol * np.abs(xn.real)) | (hi - lo <= tol * hi)
        x = np.where(active | polishing, xn, x)
        done = done | (active & small)
        if done.all() and not (left > 0).any():
            break
    if not done.all():
        raise ReturnMapNotConverged(int(np.nonzero(~done)[0][0]))
    sy, _ = flow_stress(p, epsbar, x, dt, Tstar)
    return x, sy


def j2_update(p, dF, be_n, epsbar_n, T_n, J_new, dt, spectral="eigh", polish=0, dT_extra=0.0):
    """Elastic predictor / radial return (Sec. 4.1, Sec. 4.2).

    dF: (n,3,3) incremental deformation gradient, be_n: (n,3,3) elastic left
    Cauchy-Green tensor, epsbar_n, T_n: (n,), J_new = det F_{n+1}.
    ``dT_extra`` (JC only): a temperature increment from elsewhere (heat
    conduction) added to T_{n+1} with the plastic heating; the flow stress
    still softens with T_n.
    Returns sigma, be_new, epsbar_new, T_new, deps.
    """
    lam, mu = lame(p["E"], p["nu"])
    K = lam + 2.0 * mu / 3.0
    slog, sexp = (sym_log_eigh, sym_exp_eigh) if spectral == "eigh" else \
        (sym_log_series, sym_exp_series)
    I = np.eye(3)
    b_tr = dF @ be_n @ np.swapaxes(dF, -1, -2)
    eps_tr = 0.5 * slog(b_tr)
    tr = np.trace(eps_tr, axis1=-2, axis2=-1)
    dev_tr = eps_tr - (tr / 3.0)[..., None, None] * I
    s_tr = 2.0 * mu * dev_tr
    q_tr = np.sqrt(1.5 * (s_tr * s_tr).sum(axis=(-1, -2)))
    Tstar = homologous_T(p, T_n)
    sy0, _ = flow_stress(p, epsbar_n, 0.0 * q_tr, dt, Tstar)
    plastic = q_tr.real > sy0.real
    deps = np.zeros_like(q_tr)
    if plastic.any():
        ip = np.nonzero(plastic)[0]
        x, _ = solve_return(p, q_tr[ip], epsbar_n[ip], Tstar[ip], dt, mu,
                            tol=p.get("rm_tol", 1e-14), max_iter=p.get("rm_max_iter", 60),
                            polish=polish)
        deps = deps.astype(x.dtype)
        deps[ip] = x
    q_safe = np.where(plastic, q_tr, 1.0)
    scale = np.where(plastic, 1.0 - 3.0 * mu * deps / q_safe, 1.0)
    # eps = eps_tr - (3/2) deps s_tr / q_tr ;  s = scale * s_tr
    eps = eps_tr - (1.5 * np.where(plastic, deps / q_safe, 0.0))[..., None, None] * s_tr
    tau = (K * tr)[..., None, None] * I + scale[..., None, None] * s_tr
    be_new = sexp(2.0 * eps)
    sigma = tau / J_new[..., None, None]
    epsbar_new = epsbar_n + deps
    if p["model"] == J2_JC:
        q_new = scale * q_tr
        T_new = T_n + dT_extra + p["chi"] * q_new * deps / (p["rho0"] * p["Cp"])
    else:
        T_new = T_n + 0.0 * deps
    return sigma, be_new, epsbar_new, T_new, deps


# ------------------------------------------------------- ductile fracture
def triaxiality(sigma):
    """Stress triaxiality eta = sigma_m / sigma_v of Cauchy stresses (n,3,3):
    mean stress over the von Mises stress (Sec. 4.2, fracture criterion; the
    printed p = lambda tr(eps^e) is read as the mean stress, K tr(eps^e) / J
    for the Hencky law).  0 where the stress deviator vanishes."""
    sm = np.trace(sigma, axis1=-2, axis2=-1) / 3.0
    dev = sigma - sm[..., None, None] * np.eye(3)
    sv = np.sqrt(1.5 * (dev * dev).sum(axis=(-1, -2)))
    return np.where(sv > 0, sm / np.where(sv > 0, sv, 1.0), 0.0)


def jc_fracture_strain(p, eta, deps, dt, T):
    """Critical equivalent plastic strain of the Johnson-Cook fracture
    criterion (Sec. 4.2): [d1 + d2 exp(d3 eta)] [1 + d4 ln(rate*)]
    [1 + d5 T*], rate* = max(deps / (dt rate0), 1) as in the flow stress and
    T* the homologous temperature clamped to [0, 1]."""
    d1, d2, d3, d4, d5 = (float(v) for v in p["jc_d"])
    ratio = deps / (dt * p["eps_dot0"])
    rate = np.log(np.where(ratio > 1.0, ratio, 1.0))
    ts = (T - p["T_r"]) / (p["T_m"] - p["T_r"])
    ts = np.clip(ts, 0.0, 1.0)
    with np.errstate(over="ignore"):   # near-hydrostatic compression: eps_f = inf
        return (d1 + d2 * np.exp(d3 * eta)) * (1.0 + d4 * rate) * (1.0 + d5 * ts)
