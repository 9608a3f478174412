"""Rigid cutting tool in contact with the workpiece nodes (Sec. 4.2,
non-penetration condition, penalty normal and stick forces, Coulomb slip).

Test infrastructure: a plain NumPy statement of the contact forces, used
only by the tests and the benchmark's CPU leg.

The tool is a rounded wedge extruded along z: the set of points within
r_t (tip radius) of a core wedge whose apex c(t) = c0 + t v is the centre of
the tip circle.  The core's faces are rays from c: the rake face straight up
(+y; rake angle 0) and the flank face along (cos a, sin a), a the clearance
angle, with outward normals n1 = (-1, 0) and n2 = (sin a, -cos a).  The
normal gap of a node is its signed distance to that surface (negative inside
the tool) and the contact normal is the outward normal at the closest point.

Readings (the paper points elsewhere for the details):

* the gap and the forces are evaluated at the node positions x_n and the tool
  position at t_n, and the contact force joins the internal force in the node
  update of the same step;
* the normal penalty force is c_N |g_N| along the contact normal, only for
  g_N < 0;
* the tangential gap is the elastic part of the relative tangential motion
  of node and tool since the node entered contact: each step adds the
  tangential part of (du_n - dt v) to the previous gap (first projected on
  the current tangent plane); the trial force -c_T g_T is kept if its size is
  at most mu times the normal force (stick), else it is scaled to that limit
  (slip, opposite to the slip direction) and the gap reset to -t_T / c_T;
  a node out of contact has zero tangential gap;
* the penalty stiffnesses of a node are limited to m_I / dt^2, the stiffness
  at which one step removes the node's whole penetration (the paper states
  the non-penetration condition, not its penalty constants): a node whose
  lumped mass is below c dt^2 (the light nodes a freed surface leaves) would
  otherwise make the explicit update unstable (the contact spring's
  frequency beyond 2 / dt); a node without mass gets no contact force.
"""
from __future__ import annotations

import numpy as np


def tool_frame(p):
    a = float(p["tool_clearance"])
    u1 = np.array([0.0, 1.0])
    u2 = np.array([np.cos(a), np.sin(a)])
    n1 = np.array([-1.0, 0.0])
    n2 = np.array([np.sin(a), -np.cos(a)])
    return u1, u2, n1, n2


def tool_gap(x, t, p):
    """Normal gap g_N (n,) and outward contact normal (n,3) of nodes x (n,3)
    against the tool at time t."""
    u1, u2, n1, n2 = tool_frame(p)
    c = np.asarray(p["tool_c"], float) + t * np.asarray(p["tool_v"], float)
    d = x[:, :2] - c[:2]
    a = d @ n1
    b = d @ n2
    inside = (a <= 0) & (b <= 0)
    s1 = np.maximum(d @ u1, 0.0)
    q1 = d - s1[:, None] * u1
    s2 = np.maximum(d @ u2, 0.0)
    q2 = d - s2[:, None] * u2
    l1 = np.sqrt((q1 * q1).sum(axis=1))
    l2 = np.sqrt((q2 * q2).sum(axis=1))
    first = l1 <= l2
    dist = np.where(first, l1, l2)
    safe = np.where(dist > 0, dist, 1.0)
    n_out = np.where(first[:, None], q1, q2) / safe[:, None]
    n_in = np.where((a >= b)[:, None], n1, n2)
    sd = np.where(inside, np.maximum(a, b), dist)
    nrm2 = np.where(inside[:, None], n_in, n_out)
    nrm = np.zeros((x.shape[0], 3))
    nrm[:, :2] = nrm2
    return sd - float(p["tool_r"]), nrm


def tool_forces(x, du, gT, t, p, m=None):
    """Contact force (n,3) on the nodes and their new tangential gaps (n,3).
    ``m`` (n,): the nodes' lumped masses, which limit the penalty
    stiffnesses to m / dt^2 (None: no limit)."""
    g, nrm = tool_gap(x, t, p)
    pen = g < 0
    n = x.shape[0]
    cN = np.full(n, float(p["tool_cN"]))
    cT = np.full(n, float(p["tool_cT"]))
    if m is not None:
        klim = np.where(m.real > 0, m / (p["dt"] * p["dt"]), 0.0)
        cN = np.where(klim.real < cN, klim, cN)
        cT = np.where(klim.real < cT, klim, cT)
    tn = cN * np.where(pen, -g, 0.0)
    rel = du - p["dt"] * np.asarray(p["tool_v"], float)
    rel_t = rel - (rel * nrm).sum(axis=1)[:, None] * nrm
    old_t = gT - (gT * nrm).sum(axis=1)[:, None] * nrm
    trial = old_t + rel_t
    tT = -cT[:, None] * trial
    mag = np.sqrt((tT * tT).sum(axis=1))
    lim = float(p["tool_mu"]) * tn
    slip = mag > lim
    scale = np.where(slip, lim / np.where(mag > 0, mag, 1.0), 1.0)
    tT = tT * scale[:, None]
    f = np.where(pen[:, None], tn[:, None] * nrm + tT, 0.0)
    safe = np.where(cT.real > 0, cT, 1.0)
    gT_new = np.where((pen & (cT.real > 0))[:, None], -tT / safe[:, None], 0.0)
    return f, gT_new
