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
