"""Explicit heat conduction coupled through the LME shape-function gradients.

Test infrastructure: a plain float64 reference for the GPU library, used only
by the tests, the smoke check and the benchmark's CPU baseline.

The paper's chip-formation model heats the material points adiabatically
(Sec. 4.2, temperature evolution); the cutting workload adds Fourier
conduction, q = -kappa grad T, which the paper does not discretise.  Reading
adopted here (oracle and GPU alike):

* the temperature stays a material-point field; for conduction it is
  projected to the nodes with the weights of the lumped mass,
  T_I = sum_p N_Ip m_p T_p / m_I (a uniform field projects exactly, by the
  partition of unity);
* at each MP the gradient comes from the LME gradients of the nodal field,
  grad T_p = sum_I T_I grad N_Ip, and the flux is q_p = -kappa grad T_p;
* the weak form of rho C_p dT/dt = -div q with no flux across the free
  surface, one integration point per MP and the lumped heat capacity
  C_p m_I, gives the nodal rate C_p m_I dT_I/dt = Q_I,
  Q_I = sum_p v_p q_p . grad N_Ip (the discretisation of the nodal residual
  equations of Sec. 2.1 applied to the heat equation);
* back at the MPs: dT_p = dt sum_I N_Ip Q_I / (C_p m_I).  A node without mass
  (in no support) has no temperature and no rate.

Staggering, in the rotated step (Alg. 1 with the assembly at the end):
h_I = sum_p N_Ip m_p T_p and Q_I are assembled with the mass and force; the
next node update forms T_I = h_I / m_I and Q_I / (C_p m_I); the next MP update
applies dT_p with the shape functions of step n (as for x_p and dF), adds it to
T_{n+1} with the plastic heating (the flow stress still softens with T_n),
and computes the new flux from the T_I it gathered.  The flux assembled at the
end of a step is thus the one of that step's MP update: conduction acts on the
field of the step before (an explicit two-level scheme, stable for
dt lambda_max < 1 instead of 2; the conduction time scale of the workloads is
far longer than a step).  Since sum_I grad N_Ip = 0, conduction alone keeps
sum_p m_p C_p T_p exactly (to round-off).
"""
from __future__ import annotations

import numpy as np


def assemble_heat(st, mp_of_pair, n_nodes):
    """h_I = sum_p N_Ip m_p T_p and Q_I = sum_p v_p q_p . grad N_Ip, summed per
    node in ascending (MP, pair) order."""
    h = np.bincount(st.idx, weights=st.N * st.mass[mp_of_pair] * st.T[mp_of_pair],
                    minlength=n_nodes)
    qd = st.vol[mp_of_pair] * np.einsum("qi,qi->q", st.q[mp_of_pair], st.dN)
    Q = np.bincount(st.idx, weights=qd, minlength=n_nodes)
    return h, Q


def nodal_fields(m, h, Q, Cp):
    """Nodal temperature T_I = h_I / m_I and rate Q_I / (C_p m_I); 0 without
    mass."""
    has = m > 0
    ms = np.where(has, m, 1.0)
    return np.where(has, h / ms, 0.0), np.where(has, Q / (Cp * ms), 0.0)


def mp_terms(offsets, idx, N, dN, T_nodes, rate_nodes, dt, segsum):
    """grad T_p = sum_I T_I grad N_Ip and dT_p = dt sum_I N_Ip rate_I with the
    shape functions of step n (``segsum`` sums each MP's pairs in order)."""
    tI = T_nodes[idx]
    grad = np.stack([segsum(tI * dN[:, j], offsets) for j in range(3)], axis=1)
    dT = dt * segsum(N * rate_nodes[idx], offsets)
    return grad, dT
