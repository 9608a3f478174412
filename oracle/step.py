"""One explicit OTM step (Alg. 1) on the CPU in float64.

State at the start of step n -> n+1 holds nodal positions x_I, displacement
increments du_I, lumped masses m_I and nodal forces f_I of step n, and at
the material points x_p, volume v_p, mass m_p, LME multiplier, F, b^e,
epsbar, T, Cauchy stress sigma, the support lists and N, grad N at x_p,n.
Alg. 1 is taken in rotated order: the mass/force assembly of its step 1 is
done at the end of the previous step (and once at t = 0), so that

  1. nodes:       du <- du + dt^2 f / m; x* = x + du; wall projection;
                  x <- x*                     (central difference, nodal
                                               equilibrium and position update
                                               equations; Sec. 4.1 contact)
  2. MP position: x_p <- sum_I N_I,n x_I,n+1  (MP coordinate equation)
  3. kinematics:  dF = 1 + sum_I du_I (x) grad N_I,n ; F <- dF F ;
                  v_p <- det(dF) v_p          (deformation gradient and
                                               volume equations)
  4. constitutive update                      (Sec. 4.1 / 4.2)
  5. search of the support domains            (Alg. 3)
  6. LME shape functions                      (Sec. 2.3)
  7. lumped mass and nodal force              (nodal mass and residual
       m_I = sum_p N_Ip m_p,                   equations, no body force,
       f_I = -sum_p v_p sigma_p grad N_Ip      no tractions)
           - eps sum_p N_Ip e_Ip              (stabilisation term, when
                                               eps_stab > 0)

Readings: du_0 = dt v_0 at the nodes (the central difference needs one
increment to start); the wall is rigid and frictionless: a node whose
predicted gap g = (x* - x_bar).n is negative is projected onto the plane and
its increment set to the projected motion; a node that has left every
support (zero lumped mass, zero force) keeps its increment.

Stabilisation (Sec. 2.1, stabilised residual and under-integration error):
e_Ip = [(x_I - x_p) - dF_p (x_I,prev - x_p,prev)] / |x_I,prev - x_p,prev|
with dF_p the increment of the step just taken, x_p,prev the MP position
before it and x_I,prev = x_I - du_I.  The paper gives no value for eps; it
is read as one constant with the units of a force.  At t = 0 there is no
previous configuration and no term.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import conduction, contact, lme, material, search


@dataclasses.dataclass
class State:
    x: np.ndarray
    du: np.ndarray
    m: np.ndarray
    f: np.ndarray
    xp: np.ndarray
    vol: np.ndarray
    mass: np.ndarray
    lam: np.ndarray
    F: np.ndarray
    be: np.ndarray
    epsbar: np.ndarray
    T: np.ndarray
    sigma: np.ndarray
    offsets: np.ndarray
    idx: np.ndarray
    N: np.ndarray
    dN: np.ndarray
    n: int = 0
    # MP positions before and deformation-gradient increment of the last
    # MP update (None before the first step)
    xp_prev: np.ndarray = None
    dF: np.ndarray = None
    # chip formation (Sec. 4.2): MPs that met the fracture criterion (carry
    # no stress from then on), tangential contact gaps of the nodes and the
    # time of the state (moves the tool)
    failed: np.ndarray = None
    gT: np.ndarray = None
    clock: float = 0.0
    # heat conduction (kappa > 0): MP heat flux of the last MP update, the
    # nodal sums h_I, Q_I of the last assembly and the nodal temperature and
    # rate formed from them by the node update
    q: np.ndarray = None
    node_events: tuple = (0, 0)
    heat_h: np.ndarray = None
    heat_Q: np.ndarray = None
    T_nodes: np.ndarray = None
    rate_nodes: np.ndarray = None

    def copy(self):
        return State(**{k: (v.copy() if isinstance(v, np.ndarray) else v)
                        for k, v in dataclasses.asdict(self).items()})


# ------------------------------------------------------------------ pieces
def assemble(st, p):
    """Lumped nodal mass and internal force (nodal mass / residual equations),
    summed per node in ascending (MP, pair) order."""
    n_nodes = st.x.shape[0]
    mp_of_pair = np.repeat(np.arange(st.xp.shape[0]), np.diff(st.offsets))
    m = np.bincount(st.idx, weights=(st.N * st.mass[mp_of_pair]).real, minlength=n_nodes)
    if np.iscomplexobj(st.N):
        m = m + 1j * np.bincount(st.idx, weights=(st.N * st.mass[mp_of_pair]).imag,
                                 minlength=n_nodes)
    # f_I,i = - sum_p v_p sigma_p,ij dN_Ip,j
    contrib = -st.vol[mp_of_pair, None] * np.einsum("qij,qj->qi", st.sigma[mp_of_pair], st.dN)
    eps = p.get("eps_stab", 0.0)
    if eps != 0.0 and st.xp_prev is not None:
        contrib = contrib - eps * st.N[:, None] * underintegration_error(st, mp_of_pair)
    f = np.zeros((n_nodes, 3), dtype=contrib.dtype)
    for i in range(3):
        f[:, i] = np.bincount(st.idx, weights=contrib[:, i].real, minlength=n_nodes)
        if np.iscomplexobj(contrib):
            f[:, i] = f[:, i] + 1j * np.bincount(st.idx, weights=contrib[:, i].imag,
                                                 minlength=n_nodes)
    st.m, st.f = m, f
    if st.q is not None:
        st.heat_h, st.heat_Q = conduction.assemble_heat(st, mp_of_pair, n_nodes)


def underintegration_error(st, mp_of_pair):
    """e_Ip per pair (stabilisation term, Sec. 2.1): the change of the pair's
    relative position not explained by the MP's deformation-gradient
    increment, over the pair's previous distance."""
    d = st.x[st.idx] - st.xp[mp_of_pair]
    d_prev = (st.x - st.du)[st.idx] - st.xp_prev[mp_of_pair]
    mapped = np.einsum("qij,qj->qi", st.dF[mp_of_pair], d_prev)
    dist = np.sqrt((d_prev * d_prev).sum(axis=1))
    return (d - mapped) / dist[:, None]


def node_update(st, p):
    """Central difference with lumped mass, then the rigid-wall projection."""
    dt = p["dt"]
    f = st.f
    if p.get("tool"):
        # rigid tool: penalty contact force at x_n, tool at t_n
        fc, st.gT = contact.tool_forces(st.x, st.du, st.gT, st.clock, p, st.m)
        f = f + fc
        st.clock = st.clock + dt
    # a node outside every support has no lumped mass and no force: it keeps
    # its increment (the central difference applies to nodes with mass)
    has_mass = st.m.real > 0
    m_safe = np.where(has_mass, st.m, 1.0)
    du = st.du + np.where(has_mass[:, None], dt * dt * f / m_safe[:, None], 0.0)
    xs = st.x + du
    if p["wall"]:
        nrm = np.asarray(p["wall_n"], float)
        g = (xs - np.asarray(p["wall_x"], float)) @ nrm
        hit = g.real < 0
        xs = np.where(hit[:, None], xs - g[:, None] * nrm[None, :], xs)
        du = np.where(hit[:, None], xs - st.x, du)
    st.du = du
    st.x = xs
    if st.q is not None:
        st.T_nodes, st.rate_nodes = conduction.nodal_fields(st.m, st.heat_h, st.heat_Q, p["Cp"])


def mp_update(st, p):
    """MP position, incremental deformation gradient, F, volume and the
    constitutive update, all with the shape functions of step n."""
    n_mp = st.xp.shape[0]
    xI = st.x[st.idx]
    duI = st.du[st.idx]
    xp = np.zeros((n_mp, 3), dtype=np.result_type(st.N, xI))
    for i in range(3):
        xp[:, i] = _segsum(st.N * xI[:, i], st.offsets)
    dF = np.broadcast_to(np.eye(3), (n_mp, 3, 3)).astype(np.result_type(duI, st.dN))
    for i in range(3):
        for j in range(3):
            dF[:, i, j] = dF[:, i, j] + _segsum(duI[:, i] * st.dN[:, j], st.offsets)
    F_new = dF @ st.F
    J_dF = material.det3(dF)
    # failed MPs carry nothing, so their inversion does not matter
    bad = (J_dF.real <= 0) if st.failed is None else (J_dF.real <= 0) & ~st.failed
    if np.any(bad):
        raise FloatingPointError("inverted material point (det dF <= 0) at "
                                 f"{int(np.nonzero(bad)[0][0])}")
    st.vol = J_dF * st.vol
    st.xp_prev, st.dF = st.xp, dF
    st.xp = xp
    J_new = material.det3(F_new)
    dTc, grad = 0.0, None
    if st.q is not None:
        # conduction with the shape functions of step n and the nodal field
        # of the node update
        grad, dTc = conduction.mp_terms(st.offsets, st.idx, st.N, st.dN, st.T_nodes,
                                        st.rate_nodes, p["dt"], _segsum)
    if p["model"] == material.NEOHOOKE:
        st.sigma = material.neo_hooke_cauchy(F_new, p["E"], p["nu"])
    elif st.failed is None:
        sig, be, eb, T, _ = material.j2_update(p, dF, st.be, st.epsbar, st.T, J_new, p["dt"],
                                               spectral=p.get("spectral", "eigh"),
                                               polish=p.get("polish", 0), dT_extra=dTc)
        st.sigma, st.be, st.epsbar, st.T = sig, be, eb, T
    else:
        _update_with_fracture(st, p, dF, J_new, dTc)
    if grad is not None:
        st.q = -p["kappa"] * grad
    st.F = F_new


def _update_with_fracture(st, p, dF, J_new, dTc=0.0):
    """The J2 update of the MPs that have not failed, then the Johnson-Cook
    fracture criterion (Sec. 4.2): an MP whose equivalent plastic strain is
    positive and at least the critical strain at its stress triaxiality, rate
    and temperature fails.  Readings: an MP that never yielded does not
    fracture (ductile fracture follows plastic flow); a failed MP carries no
    stress from then on (it is eroded) but keeps its mass, so the lumped mass
    is conserved, and its b^e, epsbar and T stay as they were (but for the
    conduction increment dTc, which every MP takes: a failed MP still holds
    heat)."""
    alive = np.nonzero(~st.failed)[0]
    sigma = np.zeros_like(st.sigma, dtype=np.result_type(st.sigma, dF))
    be = st.be.astype(sigma.dtype)
    eb = st.epsbar.astype(sigma.dtype)
    dTc = np.broadcast_to(np.asarray(dTc), st.T.shape)
    T = (st.T + dTc).astype(sigma.dtype)
    if alive.size:
        s_a, be_a, eb_a, T_a, de_a = material.j2_update(
            p, dF[alive], st.be[alive], st.epsbar[alive], st.T[alive], J_new[alive], p["dt"],
            spectral=p.get("spectral", "eigh"), polish=p.get("polish", 0),
            dT_extra=dTc[alive])
        eta = material.triaxiality(s_a.real)
        ef = material.jc_fracture_strain(p, eta, de_a.real, p["dt"], T_a.real)
        newly = (eb_a.real > 0) & (eb_a.real >= ef)
        s_a = np.where(newly[:, None, None], 0.0, s_a)
        sigma[alive], be[alive], eb[alive], T[alive] = s_a, be_a, eb_a, T_a
        failed = st.failed.copy()
        failed[alive[newly]] = True
        st.failed = failed
    st.sigma, st.be, st.epsbar, st.T = sigma, be, eb, T


def _segsum(vals, offsets):
    """Sum of each CSR row, pairs taken in row order."""
    out = np.zeros(offsets.shape[0] - 1, dtype=vals.dtype)
    K = np.diff(offsets)
    kmax = int(K.max()) if K.size else 0
    for k in range(kmax):
        rows = np.nonzero(K > k)[0]
        out[rows] = out[rows] + vals[offsets[rows] + k]
    return out


def rebuild_lists(st, p, x_mp_real=None):
    xm = st.xp.real if x_mp_real is None else x_mp_real
    st.offsets, st.idx = search.neighbors_linked_cell(st.x.real, xm, p["r_list"],
                                                       p["cell_size"])


def shape(st, p):
    st.lam, st.N, st.dN = lme.lme_shape(st.x, st.xp, st.offsets, st.idx, p["beta"],
                                        p["lme_tol"], p["lme_max_iter"], st.lam,
                                        extra_iter=p.get("polish", 0))


# ------------------------------------------------------------------ driver
def init_state(x_nodes, x_mp, vol, mass, v0_nodes, p, lists=None):
    """t = 0: F = b^e = 1, epsbar = 0, T = T_r, sigma = 0, du = dt v0,
    support search, shape functions, and the first mass/force assembly."""
    n_mp = x_mp.shape[0]
    n_nodes = x_nodes.shape[0]
    I = np.eye(3)
    st = State(x=np.array(x_nodes, dtype=np.float64), du=p["dt"] * np.asarray(v0_nodes, float),
               m=np.zeros(n_nodes), f=np.zeros((n_nodes, 3)),
               xp=np.array(x_mp, dtype=np.float64), vol=np.array(vol, dtype=np.float64),
               mass=np.array(mass, dtype=np.float64), lam=np.zeros((n_mp, 3)),
               F=np.tile(I, (n_mp, 1, 1)), be=np.tile(I, (n_mp, 1, 1)),
               epsbar=np.zeros(n_mp), T=np.full(n_mp, float(p["T_r"])),
               sigma=np.zeros((n_mp, 3, 3)), offsets=None, idx=None, N=None, dN=None,
               failed=np.zeros(n_mp, bool) if p.get("fracture") else None,
               gT=np.zeros((n_nodes, 3)) if p.get("tool") else None,
               q=np.zeros((n_mp, 3)) if p.get("kappa", 0.0) > 0 else None)
    if lists is None:
        rebuild_lists(st, p)
    else:
        st.offsets, st.idx = lists
    shape(st, p)
    assemble(st, p)
    return st


MP_FIELDS = ("xp", "vol", "mass", "lam", "F", "be", "epsbar", "T", "sigma", "failed", "q")
NODE_FIELDS = ("x", "du", "m", "f", "gT", "heat_h", "heat_Q")


def freed_surface_nodes(st, removed, delta):
    """Nodes inserted where material was removed (the data management of
    Sec. 3.3 adds nodes; the chip-formation workload adds them at the freed
    surfaces).  Reading: a removed MP p leaves a node at x_p when every node
    of its support is farther than ``delta`` from x_p and no removed MP of
    smaller index lies within ``delta`` of it (one node where several removed
    MPs crowd together).  The node takes the MP's interpolated increment
    sum_I N_Ip du_I, so it moves on with the material it replaces.
    Distances as in the search: ((dx*dx + dy*dy) + dz*dz), compared with
    delta^2.  Returns (positions, increments) in ascending MP order."""
    d2 = delta * delta
    xs, dus = [], []
    for k, p in enumerate(removed):
        lo, hi = st.offsets[p], st.offsets[p + 1]
        nodes = st.idx[lo:hi]
        if hi > lo and search._sqdist(st.xp[p][None, :], st.x[nodes]).min() <= d2:
            continue
        if k > 0 and search._sqdist(st.xp[p][None, :], st.xp[removed[:k]]).min() <= d2:
            continue
        xs.append(st.xp[p].copy())
        du = np.zeros(3)
        for q in range(lo, hi):
            du = du + st.N[q] * st.du[st.idx[q]]
        dus.append(du)
    return np.array(xs).reshape(-1, 3), np.array(dus).reshape(-1, 3)


def delete_orphan_nodes(st):
    """Nodes in no support (after the removal of MPs no remaining MP holds
    them) leave the node set (Sec. 3.3 deletes nodes); the others keep their
    order and the support lists are renumbered.  Returns the count."""
    n = st.x.shape[0]
    keep = np.bincount(st.idx, minlength=n) > 0
    if keep.all():
        return 0
    new_id = np.cumsum(keep) - 1
    st.idx = new_id[st.idx].astype(np.int32)
    for k in NODE_FIELDS:
        if getattr(st, k) is not None:
            setattr(st, k, getattr(st, k)[keep])
    return int((~keep).sum())


def erode(st, p):
    """Erosion: the MPs that met the fracture criterion leave the body.

    Reading: Johnson-Cook fracture separates material (Sec. 4.2) and the
    data management of Sec. 3.3 removes material points from the domain; a
    removed MP takes its mass and volume with it.  The survivors keep their
    order.  With ``insert_dist`` > 0 nodes are first added at the freed
    surface (``freed_surface_nodes``, appended after the existing nodes).
    The support lists, shape functions and the lumped mass and force of what
    remains are then recomputed, as at the end of a step; with
    ``delete_orphans`` the nodes left in no support are then removed
    (``delete_orphan_nodes``).  Returns the number of MPs removed; the node
    counts go to st.node_events = (inserted, deleted)."""
    keep = ~st.failed
    removed = np.nonzero(~keep)[0]
    inserted = deleted = 0
    delta = float(p.get("insert_dist", 0.0))
    if delta > 0 and removed.size:
        xn, dun = freed_surface_nodes(st, removed, delta)
        inserted = xn.shape[0]
        if inserted:
            st.x = np.concatenate([st.x, xn])
            st.du = np.concatenate([st.du, dun])
            for k in ("m", "heat_h", "heat_Q"):
                if getattr(st, k) is not None:
                    setattr(st, k, np.concatenate([getattr(st, k), np.zeros(inserted)]))
            for k in ("f", "gT"):
                if getattr(st, k) is not None:
                    setattr(st, k, np.concatenate([getattr(st, k), np.zeros((inserted, 3))]))
    for k in MP_FIELDS + ("xp_prev", "dF"):
        if getattr(st, k) is not None:
            setattr(st, k, getattr(st, k)[keep])
    rebuild_lists(st, p)
    shape(st, p)
    assemble(st, p)
    if p.get("delete_orphans", False):
        deleted = delete_orphan_nodes(st)
    st.node_events = (inserted, deleted)
    return int((~keep).sum())


def step(st, p, lists=None):
    """One step n -> n+1 in place.  ``lists`` (offsets, idx) forces the
    support lists (frozen-list runs); otherwise they are rebuilt every
    ``rebuild_every`` steps."""
    node_update(st, p)
    mp_update(st, p)
    st.n += 1
    if lists is not None:
        st.offsets, st.idx = lists
    elif st.n % int(p["rebuild_every"]) == 0:
        rebuild_lists(st, p)
    shape(st, p)
    assemble(st, p)
    return st


def neo_hooke_energy_density(F, E, nu):
    lam, mu = material.lame(E, nu)
    J = material.det3(F)
    trb = (F * F).sum(axis=(-1, -2))
    lnJ = np.log(J)
    return 0.5 * mu * (trb - 3.0) - mu * lnJ + 0.5 * lam * lnJ ** 2


def total_energy(st, p, vol0):
    """Kinetic energy of the half-step velocity du/dt with the lumped mass
    plus the stored Neo-Hookean energy (elastic workloads)."""
    v = st.du / p["dt"]
    ke = 0.5 * (st.m * (v * v).sum(axis=1)).sum()
    pe = (vol0 * neo_hooke_energy_density(st.F, p["E"], p["nu"])).sum()
    return ke, pe
