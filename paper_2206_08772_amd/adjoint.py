"""Checkpointed reverse-mode gradients of OTM rollouts (float64, J2 models).

``OTMRollout`` is a ``torch.autograd.Function``: its forward runs N explicit
steps of libotm and keeps a copy of the state every ``k`` steps and at the
last step; its backward walks the segments in reverse, re-runs the interior
steps of each segment from its first checkpoint while keeping every state
(the tape; both ends are checkpoints), then calls ``otm_step_adjoint`` step
by step, and ends with ``otm_init_adjoint`` for the initial velocity.  Device
buffers are torch tensors; all arithmetic is in libotm.

Gradients: with respect to the hardening constants (A, B, n, C, m of the
Johnson-Cook law, or Y0, H for linear hardening) and to the initial nodal
velocity: ``OTMRollout`` takes a scalar speed scaling a fixed unit field,
``OTMRolloutField`` the whole nodal field.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import StateBar, Tape, check, lib
from .sim import Sim, _ptr, _stream

LIST_FIELDS = ("offsets", "idx", "N", "dN")
STATE_FIELDS = ("x", "du", "m", "f", "xp", "vol", "lam", "Fd", "bed", "epsbar", "T",
                "sigma") + LIST_FIELDS
POINT_FIELDS = STATE_FIELDS[:-len(LIST_FIELDS)]   # node and MP fields


def snapshot(sim):
    """Device copy of a simulation's state (one tape entry / checkpoint)."""
    return {k: getattr(sim, k).clone() for k in STATE_FIELDS}


def empty_tape(sim, n):
    """``n`` uninitialised state snapshots carved out of one device buffer
    (one allocation instead of one per field and entry)."""
    fields = [(k, getattr(sim, k)) for k in STATE_FIELDS]
    al = lambda b: (b + 255) // 256 * 256
    per = sum(al(t.numel() * t.element_size()) for _, t in fields)
    buf = torch.empty(max(n * per, 1), dtype=torch.uint8, device=sim.device)
    tape, off = [], 0
    for _ in range(n):
        entry = {}
        for k, t in fields:
            nb = t.numel() * t.element_size()
            entry[k] = buf[off:off + nb].view(t.dtype).view(t.shape)
            off += al(nb)
        tape.append(entry)
    return tape


def snapshot_into(sim, snap, fields=STATE_FIELDS):
    """Copy state fields into preallocated tensors."""
    torch._foreach_copy_([snap[k] for k in fields], [getattr(sim, k) for k in fields])


def restore(sim, snap, fields=STATE_FIELDS):
    torch._foreach_copy_([getattr(sim, k) for k in fields], [snap[k] for k in fields])


def tape_struct(snap, n_nodes, n_mp, cap):
    t = Tape()
    t.n_nodes, t.n_mp, t.pair_stride = n_nodes, n_mp, cap
    for k in ("x", "du", "m", "f", "xp", "vol", "lam", "Fd", "bed", "epsbar", "T", "sigma", "N",
              "dN"):
        setattr(t, k, _ptr(snap[k]).value)
    t.nbr_offsets = _ptr(snap["offsets"]).value
    t.nbr_idx = _ptr(snap["idx"]).value
    return t


class Bars:
    """Adjoint buffers of one state (float64, the state's layouts)."""

    def __init__(self, n_nodes, n_mp, cap, device):
        z = lambda *s: torch.zeros(*s, dtype=torch.float64, device=device)
        self.x, self.du = z(3, n_nodes), z(3, n_nodes)
        self.vol, self.Fd, self.bed = z(n_mp), z(9, n_mp), z(6, n_mp)
        self.epsbar, self.T, self.sigma = z(n_mp), z(n_mp), z(6, n_mp)
        self.N, self.dN = z(cap), z(3, cap)

    def zero_(self):
        for k in ("x", "du", "vol", "Fd", "bed", "epsbar", "T", "sigma", "N", "dN"):
            getattr(self, k).zero_()
        return self

    def struct(self):
        b = StateBar()
        for k in ("x", "du", "vol", "Fd", "bed", "epsbar", "T", "sigma", "N", "dN"):
            setattr(b, k, _ptr(getattr(self, k)).value)
        return b


def rollout_forward(sim, steps, every, rebuild_every=1):
    """Run ``steps`` steps from the initialised ``sim``, keeping a checkpoint
    every ``every`` steps, at 0 and at the last step.  Returns the checkpoint
    dict."""
    ckpt = {0: snapshot(sim)}
    for n in range(1, steps + 1):
        sim.step(rebuild=(n % rebuild_every == 0))
        if n % every == 0 or n == steps:
            ckpt[n] = snapshot(sim)
    return ckpt


def _replay(sim, ckpt, s0, s1, tape, rebuild_every):
    """Re-run the interior steps of segment [s0, s1] from checkpoint s0 into
    ``tape``; returns the segment's states s0..s1 (both ends checkpoints).
    Each re-run step writes its lists and shape functions straight into its
    tape entry (otm_step_into), so only node and MP fields are copied."""
    states = [ckpt[s0]]
    if s1 - s0 > 1:
        restore(sim, ckpt[s0], POINT_FIELDS)
        sim.use_lists(ckpt[s0])          # read by the first step's MP update only
        for n in range(s0 + 1, s1):
            entry = tape[n - s0 - 1]
            sim.step_into(entry, rebuild=(n % rebuild_every == 0))
            snapshot_into(sim, entry, POINT_FIELDS)
            states.append(entry)
    states.append(ckpt[s1])
    return states


N_THETA = 5     # A, B, n, C, m (Johnson-Cook) or Y0, H (linear hardening)


class AdjointBuffers:
    """Device buffers of one backward sweep, allocated once (before the sweep
    is timed, or once per forward): the tape of every - 1 states, the
    adjoints of two consecutive states, the adjoint workspace, the parameter
    gradient and the initial-velocity gradient."""

    def __init__(self, sim, every, steps):
        dev = sim.device
        nn, nm, cap = sim.n_nodes, sim.n_mp, sim.cap
        self.shape = (nn, nm, cap)
        self.ws_bytes = int(lib().otm_adjoint_workspace_bytes(nn, nm))
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=dev)
        self.theta = torch.zeros(N_THETA, dtype=torch.float64, device=dev)
        self.bars = (Bars(nn, nm, cap, dev), Bars(nn, nm, cap, dev))
        self.tape = empty_tape(sim, max(min(every, steps) - 1, 0))
        self.v0_bar = torch.zeros(3, nn, dtype=torch.float64, device=dev)
        self.dir_bar = torch.zeros(1, dtype=torch.float64, device=dev)


def rollout_backward(sim, ckpt, steps, every, xbar_final, rebuild_every=1, bufs=None):
    """Adjoint sweep.  ``xbar_final`` is dL/dx at the last step ([3][n_nodes]).
    Returns (theta_bar (5,), bars of state 0); both live in ``bufs`` (an
    ``AdjointBuffers``, allocated here when not given).

    Segments are taken from the last to the first.  A segment's two ends are
    checkpoints, so only its interior states are re-run, into the tape of
    every - 1 states, refilled for each segment.  The simulation's state is
    overwritten."""
    L = lib()
    nn, nm, cap = sim.n_nodes, sim.n_mp, sim.cap
    if bufs is None:
        bufs = AdjointBuffers(sim, every, steps)
    if bufs.shape != (nn, nm, cap) or len(bufs.tape) < max(min(every, steps) - 1, 0):
        raise ValueError("adjoint buffers of another simulation or checkpoint interval")
    theta = bufs.theta
    theta.zero_()
    mass = sim.mass
    nxt, cur = bufs.bars
    nxt.zero_()
    nxt.x.copy_(xbar_final)
    starts = sorted(k for k in ckpt if k < steps)
    if not starts or starts[0] != 0 or steps not in ckpt:
        raise ValueError("checkpoints must include step 0 and the last step")
    own_lists = {k: getattr(sim, k) for k in LIST_FIELDS}
    for s0 in reversed(starts):
        s1 = min(s0 + every, steps)
        if s1 not in ckpt:
            raise ValueError(f"missing checkpoint at step {s1}")
        states = _replay(sim, ckpt, s0, s1, bufs.tape, rebuild_every)
        for j in range(s1 - s0 - 1, -1, -1):
            t0 = tape_struct(states[j], nn, nm, cap)
            t1 = tape_struct(states[j + 1], nn, nm, cap)
            bn, bc = nxt.struct(), cur.struct()
            check(L.otm_step_adjoint(C.byref(t0), C.byref(t1), C.byref(sim.p), sim.dt,
                                     _ptr(mass), C.byref(bn), C.byref(bc), _ptr(theta),
                                     _ptr(bufs.ws), bufs.ws_bytes, _ptr(sim.diag), _stream()),
                  "otm_step_adjoint")
            nxt, cur = cur, nxt
    sim.use_lists(own_lists)
    sim.check_diag()
    return theta, nxt


def initial_velocity_gradient(sim, bars0, bufs, direction=None):
    """dL/dv0 per node ([3][n_nodes] device tensor in ``bufs``) from the
    adjoint of state 0 (otm_init_adjoint); with ``direction`` ([3][n_nodes]
    device tensor) also the derivative along it (a 1-element device tensor),
    else None."""
    d = _ptr(direction) if direction is not None else C.c_void_p(0)
    db = _ptr(bufs.dir_bar) if direction is not None else C.c_void_p(0)
    check(lib().otm_init_adjoint(sim.n_nodes, sim.dt, _ptr(bars0.du), _ptr(bufs.v0_bar), d, db,
                                 _stream()), "otm_init_adjoint")
    return bufs.v0_bar, (bufs.dir_bar if direction is not None else None)


def _theta_params(p, theta):
    names = ("A", "B", "n", "C", "m") if p["model"] == _lib.OTM_J2_JC else ("Y0", "H")
    th = theta.detach().double().cpu().numpy()
    if th.shape != (N_THETA,):
        raise ValueError(f"theta must hold {N_THETA} hardening constants")
    p = dict(p)
    for k, v in zip(names, th):
        p[k] = float(v)
    return p


def _forward(ctx, theta, v0, problem):
    p = _theta_params(problem["params"], theta)
    sim = Sim(problem["x_nodes"], problem["x_mp"], problem["vol_mp"], problem["mass_mp"], v0,
              p, precision="fp64", scatter=problem.get("scatter", "atomic"),
              device=problem.get("device", "cuda"))
    sim.init()
    ckpt = rollout_forward(sim, problem["steps"], problem["every"],
                           problem.get("rebuild_every", 1))
    sim.check_diag()
    ctx.sim, ctx.ckpt, ctx.problem = sim, ckpt, problem
    ctx.bufs = AdjointBuffers(sim, problem["every"], problem["steps"])
    ctx.theta_device = theta.device
    return sim.x.t().contiguous().clone()


def _backward(ctx, grad_x):
    sim, problem = ctx.sim, ctx.problem
    xbar = grad_x.to(dtype=torch.float64).t().contiguous()
    theta_bar, bars0 = rollout_backward(sim, ctx.ckpt, problem["steps"], problem["every"],
                                        xbar, problem.get("rebuild_every", 1), bufs=ctx.bufs)
    return sim, theta_bar.clone().to(ctx.theta_device), bars0


class OTMRollout(torch.autograd.Function):
    """x_final = OTMRollout.apply(theta, speed, problem).

    theta: (5,) float64 tensor of hardening constants (A, B, n, C, m for
    Johnson-Cook; Y0, H and three unused entries for linear hardening);
    speed: scalar float64 tensor scaling ``problem['v0_unit']`` (the initial
    nodal velocity is speed * v0_unit).  ``problem`` is a dict with the
    workload arrays (x_nodes, x_mp, vol_mp, mass_mp, v0_unit), ``params``
    (flat dict, including dt), ``steps``, ``every`` (checkpoint interval) and
    optional ``rebuild_every``.  Returns the final node positions
    (n_nodes, 3) on the device.  The gradient by speed is otm_init_adjoint's
    derivative along v0_unit.
    """

    @staticmethod
    def forward(ctx, theta, speed, problem):
        ctx.speed_device = speed.device
        ctx.unit = np.asarray(problem["v0_unit"], np.float64)
        return _forward(ctx, theta, float(speed) * ctx.unit, problem)

    @staticmethod
    def backward(ctx, grad_x):
        sim, theta_bar, bars0 = _backward(ctx, grad_x)
        unit = torch.as_tensor(np.ascontiguousarray(ctx.unit.T), device=sim.device)
        _, speed_bar = initial_velocity_gradient(sim, bars0, ctx.bufs, direction=unit)
        speed_bar = speed_bar.reshape(()).clone().to(ctx.speed_device)
        ctx.sim = ctx.ckpt = ctx.bufs = None
        return theta_bar, speed_bar, None


class OTMRolloutField(torch.autograd.Function):
    """x_final = OTMRolloutField.apply(theta, v0, problem): as OTMRollout,
    with the initial nodal velocity field v0 ((n_nodes, 3) float64 tensor)
    itself as the second input; its gradient is dL/dv0 per node."""

    @staticmethod
    def forward(ctx, theta, v0, problem):
        ctx.v0_device = v0.device
        return _forward(ctx, theta, v0.detach().double().cpu().numpy(), problem)

    @staticmethod
    def backward(ctx, grad_x):
        sim, theta_bar, bars0 = _backward(ctx, grad_x)
        v0_bar, _ = initial_velocity_gradient(sim, bars0, ctx.bufs)
        v0_bar = v0_bar.t().contiguous().to(ctx.v0_device)
        ctx.sim = ctx.ckpt = ctx.bufs = None
        return theta_bar, v0_bar, None
