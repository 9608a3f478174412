"""Shared helpers of the test suite (no arithmetic of the method here)."""
import numpy as np


def rel_err(a, b):
    """Relative error of a field: max |a - b| / max |b| (0 if both vanish)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.abs(b).max() if b.size else 0.0
    num = np.abs(a - b).max() if b.size else 0.0
    if den == 0.0:
        return 0.0 if num == 0.0 else np.inf
    return num / den


def oracle_fields(st, x0_nodes, xp0, T_r):
    """Fields compared between the oracle and the GPU, in the common layout.
    Positions are compared as displacements from the start."""
    return dict(u=st.x - x0_nodes, du=st.du, m=st.m, f=st.f, up=st.xp - xp0, vol=st.vol,
                lam=st.lam, Fm1=st.F - np.eye(3), be_m1=st.be - np.eye(3), sigma=st.sigma,
                epsbar=st.epsbar, dT=st.T - T_r, N=st.N, dN=st.dN)


def gpu_fields(g, x0_nodes, xp0, T_r):
    return dict(u=g["x"] - x0_nodes, du=g["du"], m=g["m"], f=g["f"], up=g["xp"] - xp0,
                vol=g["vol"], lam=g["lam"], Fm1=g["Fd"], be_m1=g["bed"], sigma=g["sigma"],
                epsbar=g["epsbar"], dT=g["T"] - T_r, N=g["N"], dN=g["dN"])


def compare(gf, of, fields=None):
    keys = fields or [k for k in of if k in gf]
    return {k: rel_err(gf[k], of[k]) for k in keys}


def step_directions(st, rng):
    """Seeded tangent directions for the one-step map, one per state field,
    each scaled to its field: symmetric for b^e and sigma (stored as six
    components), and for epsbar and T only where the MP has flowed or
    heated (epsbar > 0, T > T at rest), away from the kinks at zero flow and
    at the reference temperature."""
    def sym(a):
        return 0.5 * (a + np.swapaxes(a, -1, -2))
    n = st.xp.shape[0]
    rms = lambda a: float(np.sqrt(np.mean(np.abs(a) ** 2))) or 1.0
    T0 = float(st.T.min())
    return dict(
        x=rng.standard_normal(st.x.shape) * rms(st.du),
        du=rng.standard_normal(st.du.shape) * rms(st.du),
        vol=rng.standard_normal(n) * st.vol,
        F=rng.standard_normal((n, 3, 3)) * rms(st.F - np.eye(3)),
        be=sym(rng.standard_normal((n, 3, 3))) * rms(st.be - np.eye(3)),
        epsbar=rng.standard_normal(n) * st.epsbar,
        T=rng.standard_normal(n) * (st.T - T0),
        sigma=sym(rng.standard_normal((n, 3, 3))) * rms(st.sigma),
        N=rng.standard_normal(st.N.shape) * st.N,
        dN=rng.standard_normal(st.dN.shape) * rms(st.dN),
    )
