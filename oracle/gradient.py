"""Oracle gradients of a rollout loss by complex-step differentiation.

The loss is L = 1/2 sum_I |x_I(N) - x_I^target|^2 over the node positions
after N explicit steps (Alg. 1).  Its derivatives with respect to the
Johnson-Cook constants A, B, n, C, m (Sec. 4.2 hardening law), to the initial
speed and along directions of the nodal initial velocity field are taken by
the complex-step method: a parameter is given an
imaginary part i*h (h ~ 1e-20 of its size), the whole rollout runs in complex
arithmetic, and dL/dtheta = Im L / h, exact up to round-off (no subtractive
cancellation).  The holomorphic form of the oracle is used for this: tensor
log/exp by series instead of eigen-decomposition, decisions (plastic branch,
wall contact, Armijo test, Newton stops) taken on real parts, and extra Newton
iterations after convergence so that the imaginary parts converge too.

Support lists are frozen to those of the real (nominal) trajectory: the
lists are piecewise constant in the parameters, so the derivative is taken
with the lists of the nominal run, step by step.
"""
from __future__ import annotations

import numpy as np

from . import step as S


def nominal_lists(x_nodes, x_mp, vol, mass, v0, p, steps):
    """Support lists of every step of the real trajectory (index 0: t = 0)."""
    st = S.init_state(x_nodes, x_mp, vol, mass, v0, p)
    lists = [(st.offsets.copy(), st.idx.copy())]
    for _ in range(steps):
        S.step(st, p)
        lists.append((st.offsets.copy(), st.idx.copy()))
    return lists, st


def rollout(x_nodes, x_mp, vol, mass, v0, p, steps, lists, complex_step=False):
    """Final state after ``steps`` steps with the given per-step lists."""
    st = S.init_state(np.asarray(x_nodes).real, np.asarray(x_mp).real, np.asarray(vol).real,
                      mass, np.asarray(v0).real, p, lists=lists[0])
    if complex_step:
        # the t = 0 quantities again, in complex arithmetic (only v0 or the
        # material constants carry an imaginary part)
        p = dict(p, spectral="series", polish=3)
        st.x = st.x.astype(complex)
        st.xp = st.xp.astype(complex)
        st.vol = st.vol.astype(complex)
        st.du = p["dt"] * np.asarray(v0, complex)
        for k in ("lam", "F", "be", "epsbar", "T", "sigma"):
            setattr(st, k, getattr(st, k).astype(complex))
        S.shape(st, p)
        S.assemble(st, p)
    for k in range(steps):
        S.step(st, p, lists=lists[k + 1])
    return st


def loss(st, x_target):
    d = st.x - x_target
    return 0.5 * (d * d).sum()


def complex_step_gradient(x_nodes, x_mp, vol, mass, v0, p, steps, lists, x_target,
                          params=("A", "B", "n"), v0_dirs=()):
    """dL/dtheta for the named material constants, dL/d(speed), where the
    initial nodal velocity is v0 = speed * v0_unit, and for each field d in
    ``v0_dirs`` (an (n_nodes, 3) array) the derivative of L along the initial
    velocity field d, under grads[("v0", k)]."""
    grads = {}
    for k, d in enumerate(v0_dirs):
        d = np.asarray(d, float)
        h = 1e-20 * np.abs(v0).max() / np.abs(d).max()
        st = rollout(x_nodes, x_mp, vol, mass, np.asarray(v0, complex) + 1j * h * d, p, steps,
                     lists, complex_step=True)
        grads[("v0", k)] = loss(st, x_target).imag / h
    for name in params:
        h = 1e-20 * abs(p[name])
        pc = dict(p)
        pc[name] = p[name] + 1j * h
        st = rollout(x_nodes, x_mp, vol, mass, v0, pc, steps, lists, complex_step=True)
        grads[name] = loss(st, x_target).imag / h
    speed = np.abs(v0).max()
    h = 1e-20 * speed
    v0c = np.asarray(v0, complex) * (1.0 + 1j * h / speed)
    st = rollout(x_nodes, x_mp, vol, mass, v0c, p, steps, lists, complex_step=True)
    grads["speed"] = loss(st, x_target).imag / h
    return grads


# ------------------------------------------------- one step as a state map
STEP_FIELDS = ("x", "du", "vol", "F", "be", "epsbar", "T", "sigma", "N", "dN")


def step_map(st, p, lists_next):
    """One step (Alg. 1) as a map of the state fields STEP_FIELDS: the lumped
    mass and force are assembled from the state's own N, grad N, sigma and v
    (nodal mass / residual equations), then the node update, the MP update
    with the shape functions of step n, and the shape functions of step n+1 on
    the given (frozen) lists.  Returns a new State; ``st`` is not changed."""
    s = st.copy()
    S.assemble(s, p)
    S.node_update(s, p)
    S.mp_update(s, p)
    s.offsets, s.idx = lists_next
    S.shape(s, p)
    return s


def step_jvp(st, p, lists_next, direction=None, param=None):
    """Directional derivative of step_map by complex step.  ``direction`` maps
    some of STEP_FIELDS to tangent arrays of their shapes; ``param`` names a
    material constant to differentiate by (per unit of that constant).
    Returns {field: derivative array} for every field in STEP_FIELDS."""
    pc = dict(p, spectral="series", polish=3)
    s = st.copy()
    for k in STEP_FIELDS + ("xp", "lam", "m", "f"):
        setattr(s, k, np.asarray(getattr(s, k), complex))
    h = 1e-20
    if direction:
        for k, d in direction.items():
            setattr(s, k, getattr(s, k) + 1j * h * np.asarray(d, float))
    if param is not None:
        h = 1e-20 * abs(p[param])
        pc[param] = p[param] + 1j * h
    out = step_map(s, pc, lists_next)
    return {k: np.asarray(getattr(out, k)).imag / h for k in STEP_FIELDS}
