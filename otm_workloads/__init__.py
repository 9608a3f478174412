"""Seeded synthetic workloads for the explicit OTM step (inputs only).

This module only builds inputs: a jittered node lattice, the tetrahedra of its
hex cells, one material point (MP) at each tet centroid with the tet volume,
the nodal initial velocity and the material constants.  It holds none of the
method's arithmetic and is shared, as plain NumPy arrays, by the CPU oracle
and by the GPU path.

The paper's two benchmarks (Taylor rod impact, Sec. 4.1; serrated chip
formation, Sec. 4.2) come with meshes and parameter tables that are not
published with it, so every workload here is a same-shape stand-in:

* nodes on the lattice (i h, j h, k h) inside the body, each coordinate
  jittered by U(-0.1 h, 0.1 h) in one seeded draw of shape (n_nodes, 3) in
  (k, j, i) order (z slowest), then numbered in Z-order (Morton order) of
  their lattice index;
* every hex cell whose 8 corners are present is split into the 6 Kuhn tets
  around its (0,0,0)-(1,1,1) diagonal; lattice points that are the corner of
  no such cell are dropped (they would be nodes without mass);
* one MP per tet at the centroid, volume |det| / 6, mass rho0 * volume,
  ordered by hex cell, the hex cells in Z-order (Morton order) of their
  lattice index, then by tet index (so any run of consecutive MPs is a compact
  brick of the body).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Kuhn split of the unit cube: corner bit 1 = +x, bit 2 = +y, bit 4 = +z.
KUHN_TETS = ((0, 1, 3, 7), (0, 1, 5, 7), (0, 2, 3, 7),
             (0, 2, 6, 7), (0, 4, 5, 7), (0, 4, 6, 7))

MODEL_NEOHOOKE = 0
MODEL_J2_JC = 1
MODEL_J2_LINEAR = 2


@dataclasses.dataclass
class Material:
    model: int
    E: float
    nu: float
    rho0: float
    # Johnson-Cook flow stress (Sec. 4.2, JC hardening law)
    A: float = 0.0
    B: float = 0.0
    n: float = 1.0
    C: float = 0.0
    m: float = 1.0
    eps_dot0: float = 1.0
    T_r: float = 293.0
    T_m: float = 1356.0
    Cp: float = 385.0
    chi: float = 0.9          # Taylor-Quinney coefficient
    # linear isotropic hardening (Sec. 4.1 yield function)
    Y0: float = 0.0
    H: float = 0.0
    # thermal conductivity (W / (m K)); 0: adiabatic, no conduction
    kappa: float = 0.0

    @property
    def lame(self):
        lam = self.E * self.nu / ((1 + self.nu) * (1 - 2 * self.nu))
        mu = self.E / (2 * (1 + self.nu))
        return lam, mu

    @property
    def wave_speed(self):
        lam, mu = self.lame
        return math.sqrt((lam + 2 * mu) / self.rho0)


@dataclasses.dataclass
class Workload:
    name: str
    h: float
    x_nodes: np.ndarray     # (n_nodes, 3) float64, jittered reference positions
    X_nominal: np.ndarray   # (n_nodes, 3) float64, unjittered lattice points
    x_mp: np.ndarray        # (n_mp, 3) float64, tet centroids
    vol_mp: np.ndarray      # (n_mp,) tet volumes
    mass_mp: np.ndarray     # (n_mp,) rho0 * volume
    v0_nodes: np.ndarray    # (n_nodes, 3) initial nodal velocity
    material: Material
    dt: float
    steps: int
    gamma: float = 4.0
    shape_cut: float = 1e-6
    skin: float = 0.0
    rebuild_every: int = 1
    wall: bool = False
    wall_x: tuple = (0.0, 0.0, 0.0)
    wall_n: tuple = (0.0, 0.0, 1.0)
    # Johnson-Cook fracture constants d1..d5 (chip formation, fracture
    # criterion), or None
    fracture: tuple = None
    # rigid cutting tool (chip formation, contact): dict with c0 (centre of the
    # tip circle at t = 0), v (velocity), r (tip radius), clearance (rad),
    # cN, cT (penalty stiffnesses, N/m), mu (Coulomb coefficient), or None
    tool: dict = None
    # node management at erosion: nodes added at the freed surface within
    # this distance rule (0: none) and nodes in no support deleted
    insert_dist: float = 0.0
    delete_orphans: bool = False

    @property
    def n_nodes(self):
        return self.x_nodes.shape[0]

    @property
    def n_mp(self):
        return self.x_mp.shape[0]

    @property
    def beta(self):
        # beta = gamma / h^2 (Sec. 2.3)
        return self.gamma / self.h ** 2

    @property
    def r_cut(self):
        # support radius at which the Gaussian prior exp(-beta r^2) drops to
        # the shape-value cut: r = h sqrt(-ln(cut) / gamma)
        return self.h * math.sqrt(-math.log(self.shape_cut) / self.gamma)

    @property
    def r_list(self):
        return self.r_cut + self.skin


def _morton3(i, j, k):
    """Morton (Z-order) code of non-negative integer lattice indices: their
    bits interleaved, 21 bits each."""
    def spread(v):
        v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
        v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
        v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
        v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
        return v
    return spread(i) | (spread(j) << np.uint64(1)) | (spread(k) << np.uint64(2))


def _lattice_body(ijk_ranges, inside, h, seed, clamp_z0=False, clamp_x0=False,
                  hex_order="morton", node_order="morton", clamp_x1=None):
    """Lattice nodes inside a body, their jitter, the hex cells and tets.

    ``inside(i, j, k)`` receives integer index arrays and returns a mask.
    Returns (x_nodes, X_nominal, x_mp, vol_mp).
    """
    (i0, i1), (j0, j1), (k0, k1) = ijk_ranges
    ni, nj, nk = i1 - i0 + 1, j1 - j0 + 1, k1 - k0 + 1
    kk, jj, ii = np.meshgrid(np.arange(k0, k1 + 1), np.arange(j0, j1 + 1),
                             np.arange(i0, i1 + 1), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    mask = inside(ii, jj, kk)
    X = np.stack([ii[mask], jj[mask], kk[mask]], axis=1).astype(np.float64) * h
    rng = np.random.default_rng(seed)
    jit = rng.uniform(-0.1 * h, 0.1 * h, size=X.shape)   # drawn in (k, j, i) order
    if node_order == "morton":
        # nodes numbered in Z-order of their lattice index, like the hexes:
        # the nodes a run of consecutive MPs touches sit close together
        order = np.argsort(_morton3(ii[mask] - i0, jj[mask] - j0, kk[mask] - k0), kind="stable")
    else:
        order = np.arange(X.shape[0])
    X, jit = X[order], jit[order]
    rank = np.empty(order.size, dtype=np.int64)
    rank[order] = np.arange(order.size)
    node_id = np.full(mask.shape[0], -1, dtype=np.int64)
    node_id[mask] = rank
    node_id = node_id.reshape(nk, nj, ni)
    x = X + jit
    if clamp_z0:
        x[:, 2] = np.maximum(x[:, 2], 0.0)
    if clamp_x0:
        x[:, 0] = np.maximum(x[:, 0], 0.0)
    if clamp_x1 is not None:
        x[:, 0] = np.minimum(x[:, 0], clamp_x1)

    # hex cells with all 8 corners present, in (k, j, i) order
    corners = []
    for c in range(8):
        di, dj, dk = c & 1, (c >> 1) & 1, (c >> 2) & 1
        corners.append(node_id[dk:nk - 1 + dk, dj:nj - 1 + dj, di:ni - 1 + di].ravel())
    corners = np.stack(corners, axis=1)
    full = (corners >= 0).all(axis=1)
    corners = corners[full]
    if hex_order == "morton":
        # hexes (and so their MPs) in Z-order of their lattice index: any run
        # of consecutive MPs is a compact brick of the body
        kk, jj, ii = np.meshgrid(np.arange(nk - 1), np.arange(nj - 1), np.arange(ni - 1),
                                 indexing="ij")
        code = _morton3(ii.ravel()[full], jj.ravel()[full], kk.ravel()[full])
        corners = corners[np.argsort(code, kind="stable")]
    tet_nodes = corners[:, np.array(KUHN_TETS)]          # (n_hex, 6, 4)
    tet_nodes = tet_nodes.reshape(-1, 4)
    # lattice points that belong to no complete hex cell would carry no mass
    # of their own: keep only the corners of the tets (order preserved)
    used = np.zeros(x.shape[0], dtype=bool)
    used[tet_nodes.ravel()] = True
    renum = np.cumsum(used) - 1
    x, X = x[used], X[used]
    tet_nodes = renum[tet_nodes]
    p = x[tet_nodes]                                       # (n_mp, 4, 3)
    x_mp = p.mean(axis=1)
    e = p[:, 1:, :] - p[:, :1, :]
    vol = np.abs(np.linalg.det(e)) / 6.0
    return x, X, x_mp, vol


def elastic_cube(n=10, h=1.0, seed=0, steps=10):
    """Elastic cube: n^3 node lattice, Neo-Hookean E=200, nu=0.3, rho=1,
    v_x = 0.01 sin(pi X / L) with X the nominal x and L = (n - 1) h."""
    L = (n - 1) * h
    x, X, x_mp, vol = _lattice_body(((0, n - 1),) * 3,
                                    lambda i, j, k: np.ones(i.shape, bool), h, seed)
    mat = Material(MODEL_NEOHOOKE, E=200.0, nu=0.3, rho0=1.0)
    v0 = np.zeros_like(x)
    v0[:, 0] = 0.01 * np.sin(np.pi * X[:, 0] / L)
    dt = 0.1 * h / mat.wave_speed
    return Workload("elastic_cube", h, x, X, x_mp, vol, mat.rho0 * vol, v0, mat, dt, steps)


def heat_bar(n=(21, 3, 3), h=1.0, seed=0, kappa=1.0, rho0=1.0, Cp=1.0, dt=0.02, steps=500):
    """A bar at rest for heat conduction: an (nx, ny, nz) node lattice of
    spacing h, a J2/JC material that never yields (A far above any stress;
    nothing moves, so the stress stays 0), thermal conductivity kappa,
    density rho0 and heat capacity Cp (diffusivity kappa / (rho0 Cp)), no
    velocity.  The initial temperature field is the caller's."""
    nx, ny, nz = n
    x, X, x_mp, vol = _lattice_body(((0, nx - 1), (0, ny - 1), (0, nz - 1)),
                                    lambda i, j, k: np.ones(i.shape, bool), h, seed)
    mat = Material(MODEL_J2_JC, E=200.0, nu=0.3, rho0=rho0, A=1e30, B=0.0, n=1.0, C=0.0,
                   m=1.0, T_r=0.0, T_m=1e6, Cp=Cp, chi=0.0, kappa=kappa)
    return Workload("heat_bar", h, x, X, x_mp, vol, rho0 * vol, np.zeros_like(x), mat, dt,
                    steps)


def jc_params(seed):
    """Johnson-Cook constants drawn from copper-like ranges (Pa, SI units)."""
    rng = np.random.default_rng(seed)
    return dict(A=rng.uniform(80e6, 100e6), B=rng.uniform(250e6, 320e6),
                n=rng.uniform(0.25, 0.35), C=rng.uniform(0.02, 0.03),
                m=rng.uniform(1.0, 1.1))


def taylor_rod(h, seed, radius=3.2e-3, length=21.12e-3, speed=190.0, steps=100,
               model=MODEL_J2_JC, skin_h=0.0, rebuild_every=1, name="taylor_rod",
               material=None, dt=None, hex_order="morton"):
    """Cylinder of radius R and length L (z axis) on a jittered lattice,
    flying at -speed along z into a rigid frictionless wall z = 0.

    Copper elastic constants of the paper's Taylor rod (Sec. 4.1), JC flow
    stress drawn from ``seed``, Taylor-Quinney 0.9.
    """
    nr = int(math.floor(radius / h))
    nz = int(math.floor(length / h))

    def inside(i, j, k):
        return (i * h) ** 2 + (j * h) ** 2 <= radius ** 2

    x, X, x_mp, vol = _lattice_body(((-nr, nr), (-nr, nr), (0, nz)), inside, h, seed,
                                    clamp_z0=True, hex_order=hex_order)
    if material is None:
        material = Material(model, E=117e9, nu=0.35, rho0=8930.0, chi=0.9,
                            T_r=293.0, T_m=1356.0, Cp=385.0, eps_dot0=1.0,
                            Y0=400e6, H=100e6, **jc_params(seed))
    v0 = np.zeros_like(x)
    v0[:, 2] = -speed
    if dt is None:
        dt = 0.1 * h / material.wave_speed
    return Workload(name, h, x, X, x_mp, vol, material.rho0 * vol, v0, material, dt, steps,
                    skin=skin_h * h, rebuild_every=rebuild_every, wall=True)


def ti_params(seed):
    """Ti-alloy-like Johnson-Cook flow and fracture constants drawn from
    ``seed`` (Pa, SI units): the chip-formation study takes its values from a
    reference that is not published with it."""
    rng = np.random.default_rng(seed)
    flow = dict(A=rng.uniform(860e6, 1100e6), B=rng.uniform(330e6, 700e6),
                n=rng.uniform(0.30, 0.60), C=rng.uniform(0.012, 0.035),
                m=rng.uniform(0.8, 1.1))
    frac = (rng.uniform(-0.09, 0.05), rng.uniform(0.25, 0.35), rng.uniform(-0.5, -0.45),
            rng.uniform(0.014, 0.03), rng.uniform(3.5, 3.9))
    return flow, frac


def cutting_slab(h=2e-6, seed=7, length=300e-6, height=120e-6, layers=3, depth=100e-6,
                 speed=5.0, tip_radius=2e-6, clearance_deg=7.0, engage=0.0, steps=2000,
                 dt=1e-10, name="cutting_slab", fracture=None, flat_face=False):
    """Orthogonal cutting (Sec. 4.2): a workpiece of length x height
    (x, y) and ``layers`` node layers through the thickness (z), a rigid tool
    of tip radius 2 um and rake angle 0 moving at -speed along x with the
    cutting depth ``depth`` below the top face, the workpiece held at x = 0
    by the frictionless wall.  Ti-alloy-like elastic constants and
    Taylor-Quinney coefficient, the paper's T_m = 1630 C and T_r = 25 C,
    Johnson-Cook flow and fracture constants from ``seed``; Coulomb
    friction 0.8; normal and tangential penalties E h.  ``engage`` moves the
    tool that far into the workpiece at t = 0; ``flat_face`` clamps the
    jittered nodes to x <= length, so that a tool starting at the face
    touches it without overlap."""
    ni = int(round(length / h))
    nj = int(round(height / h))
    x, X, x_mp, vol = _lattice_body(((0, ni), (0, nj), (0, layers - 1)),
                                    lambda i, j, k: np.ones(i.shape, bool), h, seed,
                                    clamp_x0=True, clamp_x1=length if flat_face else None)
    flow, frac = ti_params(seed)
    mat = Material(MODEL_J2_JC, E=113.8e9, nu=0.342, rho0=4430.0, chi=0.9,
                   T_r=298.15, T_m=1903.15, Cp=580.0, eps_dot0=1.0, **flow)
    v0 = np.zeros_like(x)
    tool = dict(c0=(length + tip_radius - engage, height - depth + tip_radius, 0.0),
                v=(-speed, 0.0, 0.0), r=tip_radius, clearance=math.radians(clearance_deg),
                cN=mat.E * h, cT=mat.E * h, mu=0.8)
    return Workload(name, h, x, X, x_mp, vol, mat.rho0 * vol, v0, mat, dt, steps,
                    wall=True, wall_x=(0.0, 0.0, 0.0), wall_n=(1.0, 0.0, 0.0),
                    fracture=tuple(frac) if fracture is None else tuple(fracture), tool=tool)


def cutting_slab_5m(h=4.64e-6, seed=11, steps=500):
    """Orthogonal cutting at the scale of a production run: a 2 x 1 x 0.05 mm
    workpiece (431 x 216 x 12 node lattice, 1.12M nodes and 6.14M MPs),
    the rigid tool (rake angle 0, tip radius 2 um, clearance 7 deg) at 5 m/s
    with 0.1 mm depth of cut, starting 0.1 um (2 % of h) into the workpiece's
    face (made flat: the jitter would otherwise put nodes up to 0.46 um inside
    the tool at t = 0, which the penalty contact fires off at ~10^3 m/s),
    dt = 1e-10 s, 500 steps, Ti-alloy-like flow constants from ``seed``, heat
    conduction with the Ti-alloy conductivity 6.7 W/(m K), and low fracture
    constants d = (0, 0.005, -0.5, 0.014, 3.7) so that MPs ahead of the tool
    fail and are removed within the run (the real constants would need far
    more steps; in 500 steps the tool advances 0.25 um, and the initial
    engagement is what makes the MPs at the tool yield and fail within the
    run); nodes are added at the freed surface (insert_dist = h / 2) and
    nodes left in no support deleted.  Erosion leaves light nodes at the
    tool tip; the contact penalty limited by the nodal mass keeps them
    stable (without that limit the run blew up a few tens of steps after
    the second erosion)."""
    w = cutting_slab(h=h, seed=seed, length=2e-3, height=1e-3, layers=12, depth=0.1e-3,
                     speed=5.0, steps=steps, dt=1e-10, name="cutting_slab_5m",
                     fracture=(0.0, 0.005, -0.5, 0.014, 3.7), flat_face=True,
                     engage=0.1e-6)
    w.material.kappa = 6.7
    w.insert_dist = 0.5 * h
    w.delete_orphans = True
    return w


def config_by_name(name):
    """The named workloads.

    elastic_cube   10^3 nodes, 4374 MPs, Neo-Hookean, 10 steps
    taylor_rod     ~202k nodes / ~1.13M MPs, J2/JC + heating + wall, 100 steps
    taylor_rod_xl  ~2.0M nodes / ~11.6M MPs, lists rebuilt every 10 steps with
                   a 0.1 h skin, 200 steps
    adjoint_rod    ~50k nodes / ~268k MPs, 200 steps (gradient workload)
    small_rod      ~0.8k nodes / ~3.5k MPs rod for long oracle trajectories
    paper_rod      the Taylor rod of Sec. 4.1 at the paper's size: L = 32.4 mm,
                   R = 3.2 mm, 227 m/s, linear hardening Y0 = 400 MPa,
                   H = 100 MPa, dt = 4e-9 s, 2000 steps; h = 0.55 mm gives
                   5,959 nodes / 27,840 MPs (the paper's mesh: 5,966 / 28,423)
    cutting_slab   the chip-formation workpiece of Sec. 4.2 at the paper's size:
                   300 x 120 um, h = 2 um, 3 node layers: 27,633 nodes /
                   108,000 MPs (the paper's model: 27,417 / 107,975), rigid
                   tool with 2 um tip radius, 0 rake, 100 um depth of cut,
                   starting 0.25 um clear of the face at 20 m/s (the paper
                   gives no cutting speed), JC flow and fracture,
                   dt = 1e-10 s, 2000 steps
    small_cut      a 40 x 24 um piece of the same slab (h = 2 um) with the tool
                   0.2 um clear of it, at 50 m/s, and a low fracture strain
                   (parity tests: contact, friction and fracture within steps)
    """
    if name == "elastic_cube":
        return elastic_cube()
    if name == "taylor_rod":
        return taylor_rod(h=0.15033e-3, seed=1, steps=100)
    if name == "cutting_slab_5m":
        return cutting_slab_5m()
    if name == "taylor_rod_xl":
        return taylor_rod(h=0.06978e-3, seed=2, steps=200, skin_h=0.1, rebuild_every=10,
                          name="taylor_rod_xl")
    if name == "adjoint_rod":
        return taylor_rod(h=0.23863e-3, seed=3, steps=200, name="adjoint_rod")
    if name == "small_rod":
        return taylor_rod(h=0.8e-3, seed=5, radius=3.2e-3, length=10.4e-3, steps=100,
                          name="small_rod")
    if name == "paper_rod":
        return taylor_rod(h=0.55e-3, seed=6, radius=3.2e-3, length=32.4e-3, speed=227.0,
                          steps=2000, model=MODEL_J2_LINEAR, name="paper_rod", dt=4e-9)
    if name == "cutting_slab":
        return cutting_slab(speed=20.0, engage=-0.25e-6)
    if name == "small_cut":
        return cutting_slab(length=40e-6, height=24e-6, depth=16e-6, speed=50.0,
                            engage=-0.2e-6, steps=60, name="small_cut",
                            fracture=(0.0, 0.005, -0.5, 0.014, 3.7))
    raise KeyError(name)


def random_cloud(n_nodes, n_mp, seed, box=1.0):
    """Uniform random nodes and MPs in a cube (search tests)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0, box, (n_nodes, 3)), rng.uniform(0, box, (n_mp, 3))


def params_from_workload(w, **over):
    """Flat parameter dict of a workload: material constants, LME locality,
    search radius and cell edge, solver tolerances, wall and time step.  Both
    the oracle and the GPU library take their parameters from this dict."""
    mat = w.material
    p = dict(model=mat.model, E=mat.E, nu=mat.nu, rho0=mat.rho0, A=mat.A, B=mat.B,
             n=mat.n, C=mat.C, m=mat.m, eps_dot0=mat.eps_dot0, T_r=mat.T_r, T_m=mat.T_m,
             Cp=mat.Cp, chi=mat.chi, Y0=mat.Y0, H=mat.H, kappa=mat.kappa,
             beta=w.beta, r_list=w.r_list, cell_size=w.r_list * 1.0001,
             lme_tol=1e-14 * w.h, lme_max_iter=50, rm_tol=1e-14, rm_max_iter=60,
             wall=bool(w.wall), wall_x=np.array(w.wall_x, float),
             wall_n=np.array(w.wall_n, float), dt=w.dt, rebuild_every=w.rebuild_every,
             fracture=w.fracture is not None,
             jc_d=np.array(w.fracture if w.fracture is not None else (0.0,) * 5, float),
             tool=w.tool is not None, insert_dist=w.insert_dist,
             delete_orphans=w.delete_orphans)
    if w.tool is not None:
        t = w.tool
        p.update(tool_c=np.array(t["c0"], float), tool_v=np.array(t["v"], float),
                 tool_r=float(t["r"]), tool_clearance=float(t["clearance"]),
                 tool_cN=float(t["cN"]), tool_cT=float(t["cT"]), tool_mu=float(t["mu"]))
    p.update(over)
    return p
