"""Python front end of libotm: device buffers (torch tensors on the current
HIP device), the caller's stream, and thin wrappers of the C entry points.

All arithmetic of the method runs inside libotm's kernels; this module only
allocates, lays out and passes pointers.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import Diag, Params, State, check, lib

SYM = ((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2))


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


def _addr(t):
    """Device address of a state array: an empty view (a body whose MPs were
    all removed) still names its allocation, which the state checks want."""
    if t is None:
        return C.c_void_p(0)
    return C.c_void_p(t.untyped_storage().data_ptr() + t.storage_offset() * t.element_size())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def soa(a, device, dtype=torch.float64):
    """(n, k) host array -> contiguous [k][n] device tensor."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).T)
    return torch.from_numpy(a).to(device=device, dtype=dtype).contiguous()


def make_params(p):
    """otm_params from a flat dict (the keys of the oracle's parameter dict)."""
    q = Params()
    q.model = int(p["model"])
    q.wall_enabled = 1 if p.get("wall", False) else 0
    for k in ("E", "nu", "rho0", "A", "B", "n", "C", "m", "eps_dot0", "T_r", "T_m", "Cp",
              "chi", "Y0", "H", "beta", "r_list", "cell_size", "lme_tol", "rm_tol"):
        setattr(q, k, float(p[k]))
    q.lme_max_iter = int(p.get("lme_max_iter", 50))
    q.rm_max_iter = int(p.get("rm_max_iter", 60))
    wx = p.get("wall_x", (0.0, 0.0, 0.0))
    wn = p.get("wall_n", (0.0, 0.0, 1.0))
    for i in range(3):
        q.wall_x[i] = float(wx[i])
        q.wall_n[i] = float(wn[i])
        q.body_force[i] = 0.0
    q.eps_stab = float(p.get("eps_stab", 0.0))
    q.kappa = float(p.get("kappa", 0.0))
    q.insert_dist = float(p.get("insert_dist", 0.0))
    q.delete_orphans = 1 if p.get("delete_orphans", False) else 0
    q.fracture = 1 if p.get("fracture", False) else 0
    q.tool_enabled = 1 if p.get("tool", False) else 0
    d = p.get("jc_d", (0.0,) * 5)
    for k in range(5):
        q.jc_d[k] = float(d[k])
    if q.tool_enabled:
        for i in range(3):
            q.tool_c[i] = float(p["tool_c"][i])
            q.tool_v[i] = float(p["tool_v"][i])
        for k in ("tool_r", "tool_clearance", "tool_cN", "tool_cT", "tool_mu"):
            setattr(q, k, float(p[k]))
    return q


class Workspace:
    def __init__(self, n_nodes, n_mp, cap, device):
        self.nbytes = int(lib().otm_workspace_bytes(n_nodes, n_mp, cap))
        self.buf = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)

    @property
    def ptr(self):
        return _ptr(self.buf)


def new_diag(device):
    d = torch.empty(C.sizeof(Diag), dtype=torch.uint8, device=device)
    check(lib().otm_diag_reset(_ptr(d), _stream()), "otm_diag_reset")
    return d


def read_diag(d):
    out = Diag()
    code = lib().otm_diag_read(_ptr(d), C.byref(out), _stream())
    return code, out


# -------------------------------------------------------------- single calls
def build_neighbors(x_nodes, x_mp, r_list, cell_size, pair_capacity=None):
    """Support lists of device positions x_nodes [3][nn], x_mp [3][np].
    Returns (offsets int64 [np+1], idx int32 [P]) device tensors."""
    dev = x_nodes.device
    nn, nm = x_nodes.shape[1], x_mp.shape[1]
    offsets = torch.empty(nm + 1, dtype=torch.int64, device=dev)
    P = C.c_int64(0)
    if pair_capacity is None:
        ws = Workspace(nn, nm, 0, dev)
        code = lib().otm_build_neighbors(nn, _ptr(x_nodes), nm, _ptr(x_mp), r_list, cell_size, 0,
                                         _ptr(offsets), C.c_void_p(0), C.byref(P), ws.ptr,
                                         ws.nbytes, _stream())
        if code not in (_lib.OTM_OK, _lib.OTM_ERR_CAPACITY):
            check(code, "otm_build_neighbors")
        pair_capacity = int(P.value)
    idx = torch.empty(max(pair_capacity, 1), dtype=torch.int32, device=dev)
    ws = Workspace(nn, nm, pair_capacity, dev)
    code = lib().otm_build_neighbors(nn, _ptr(x_nodes), nm, _ptr(x_mp), r_list, cell_size,
                                     pair_capacity, _ptr(offsets), _ptr(idx), C.byref(P), ws.ptr,
                                     ws.nbytes, _stream())
    check(code, "otm_build_neighbors")
    return offsets, idx[:P.value]


def lme_shape(x_nodes, x_mp, offsets, idx, beta, tol, max_iter=50, lam=None, precision=0,
              diag=None):
    """LME shape functions on device lists.  Returns (lam, N, dN, diag)."""
    dev = x_nodes.device
    nn, nm = x_nodes.shape[1], x_mp.shape[1]
    cap = max(int(idx.numel()), 1)
    lam = torch.zeros(3, nm, dtype=torch.float64, device=dev) if lam is None else lam
    N = torch.empty(cap, dtype=torch.float64, device=dev)
    dN = torch.empty(3, cap, dtype=torch.float64 if precision == 0 else torch.float32,
                     device=dev)
    diag = new_diag(dev) if diag is None else diag
    check(lib().otm_lme_shape(nn, _ptr(x_nodes), nm, _ptr(x_mp), _ptr(offsets), _ptr(idx), cap,
                              beta, tol, max_iter, _ptr(lam), _ptr(N), _ptr(dN), precision,
                              _ptr(diag), _stream()), "otm_lme_shape")
    P = int(idx.numel())
    return lam, N[:P], dN[:, :P], diag


# -------------------------------------------------------------- simulation
class Sim:
    """Device state of one OTM simulation.

    x_nodes (nn,3), x_mp (np,3), vol_mp, mass_mp (np,), v0_nodes (nn,3) are
    host arrays; ``params`` is a flat dict (oracle keys, including ``dt``).
    ``precision`` is "fp64", "mixed" (float32 return map and force products)
    or "mixed_storage" (float32 storage, float64 arithmetic); ``scatter``
    "atomic" or "segmented"
    (bit-reproducible).  The pair buffer is sized from a first search times
    ``capacity_margin``.  Optional parts follow ``params``: ``eps_stab`` > 0
    (stabilisation term), ``fracture`` with ``jc_d`` (Johnson-Cook fracture)
    and ``tool`` with the ``tool_*`` keys (rigid cutting tool).

        import otm_workloads as W
        w = W.config_by_name("taylor_rod")
        sim = Sim(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes,
                  W.params_from_workload(w))
        sim.init()                    # search, shape functions, assembly at t = 0
        sim.run(100)                  # otm_step x 100 on the current stream
        sim.check_diag()              # raises on any device-side failure
        f = sim.fields()              # host copies in (n, 3) / (n, 3, 3) layouts
    """

    def __init__(self, x_nodes, x_mp, vol_mp, mass_mp, v0_nodes, params, precision="fp64",
                 scatter="atomic", pair_capacity=None, capacity_margin=1.3, device="cuda",
                 node_capacity=None):
        self.device = torch.device(device)
        self.params = dict(params)
        self.p = make_params(params)
        self.dt = float(params["dt"])
        precs = {"fp64": _lib.OTM_FP64, "mixed": _lib.OTM_MIXED,
                 "mixed_storage": _lib.OTM_MIXED_STORAGE}
        if precision not in precs:
            raise ValueError(f"precision must be one of {sorted(precs)}")
        self.prec = precs[precision]
        self.mode = _lib.OTM_SCATTER_ATOMIC if scatter == "atomic" else _lib.OTM_SCATTER_SEGMENTED
        dev = self.device
        rdt = torch.float64 if self.prec == _lib.OTM_FP64 else torch.float32
        nn, nm = len(x_nodes), len(x_mp)
        self.n_nodes, self.n_mp = nn, nm
        # node arrays: room for nodes added at erosion (insert_dist > 0); each
        # array is a [k][n_nodes] view of the first k * n_nodes entries
        insert = float(params.get("insert_dist", 0.0)) > 0.0
        if node_capacity is None:
            node_capacity = nn + (max(1024, nm // 4) if insert else 0)
        self.ncap = max(int(node_capacity), nn)
        self._node_bufs = {}
        self.x = self._node_array("x", 3)
        self.x.copy_(soa(x_nodes, dev))
        self.du = self._node_array("du", 3)
        self.m = self._node_array("m", 1)
        self.f = self._node_array("f", 3)
        self.xp = soa(x_mp, dev)
        self.vol = torch.as_tensor(np.asarray(vol_mp, np.float64), device=dev).clone()
        self.mass = torch.as_tensor(np.asarray(mass_mp, np.float64), device=dev).clone()
        self.lam = torch.zeros(3, nm, dtype=torch.float64, device=dev)
        self.Fd = torch.zeros(9, nm, dtype=rdt, device=dev)
        self.bed = torch.zeros(6, nm, dtype=rdt, device=dev)
        self.epsbar = torch.zeros(nm, dtype=torch.float64, device=dev)
        self.T = torch.zeros(nm, dtype=torch.float64, device=dev)
        self.sigma = torch.zeros(6, nm, dtype=rdt, device=dev)
        # history of the stabilisation term (written by each step's MP update)
        self.stab = float(params.get("eps_stab", 0.0)) > 0.0
        self.xp_prev = torch.zeros(3, nm, dtype=torch.float64, device=dev) if self.stab else None
        self.dFm1 = torch.zeros(9, nm, dtype=torch.float64, device=dev) if self.stab else None
        # chip formation: fracture flags, tangential contact gaps, the clock
        self.fracture = bool(params.get("fracture", False))
        self.tool = bool(params.get("tool", False))
        self.failed = torch.zeros(nm, dtype=torch.int32, device=dev) if self.fracture else None
        self.tool_gt = self._node_array("tool_gt", 3) if self.tool else None
        self.clock = torch.zeros(1, dtype=torch.float64, device=dev) if self.tool else None
        # heat conduction: nodal sums h_I, Q_I of the assembly and MP fluxes
        self.cond = float(params.get("kappa", 0.0)) > 0.0
        self.heat = self._node_array("heat", 2) if self.cond else None
        self.qflux = torch.zeros(3, nm, dtype=torch.float64, device=dev) if self.cond else None
        self.offsets = torch.zeros(nm + 1, dtype=torch.int64, device=dev)
        self.v0 = soa(v0_nodes, dev)
        if pair_capacity is None:
            P = self._count_pairs()
            # even, so that the MP update can load two pairs at once
            pair_capacity = (int(P * capacity_margin) + 1024 + 1) // 2 * 2
        self.cap = int(pair_capacity)
        self.idx = torch.zeros(self.cap, dtype=torch.int32, device=dev)
        self.N = torch.zeros(self.cap, dtype=torch.float64, device=dev)
        self.dN = torch.zeros(3, self.cap, dtype=rdt, device=dev)
        self.ws = Workspace(self.ncap, nm, self.cap, dev)
        self.node_events = (0, 0)
        self.diag = new_diag(dev)
        self.st = State()
        self._fill_state()
        self.n = 0
        # bumped whenever the state's arrays move or change shape (erosion,
        # swapped lists): graphs captured before hold the old layout
        self.layout = 0

    def _node_array(self, name, comps):
        """A zeroed [comps][n_nodes] float64 view into a buffer with room for
        ``ncap`` nodes."""
        buf = torch.zeros(comps * self.ncap, dtype=torch.float64, device=self.device)
        self._node_bufs[name] = (buf, comps)
        return self._node_view(name, self.n_nodes)

    def _node_view(self, name, n):
        buf, comps = self._node_bufs[name]
        v = buf[: comps * n]
        return v if comps == 1 else v.view(comps, n)

    def _count_pairs(self):
        P = C.c_int64(0)
        ws = Workspace(self.n_nodes, self.n_mp, 0, self.device)
        code = lib().otm_build_neighbors(self.n_nodes, _ptr(self.x), self.n_mp, _ptr(self.xp),
                                         self.p.r_list, self.p.cell_size, 0, _ptr(self.offsets),
                                         C.c_void_p(0), C.byref(P), ws.ptr, ws.nbytes, _stream())
        if code not in (_lib.OTM_OK, _lib.OTM_ERR_CAPACITY):
            check(code, "otm_build_neighbors")
        return int(P.value)

    def _fill_state(self):
        s = self.st
        s.n_nodes, s.n_mp, s.pair_capacity, s.precision = self.n_nodes, self.n_mp, self.cap, self.prec
        for k in ("x", "du", "m", "f", "xp", "vol", "mass", "lam", "Fd", "bed", "epsbar", "T",
                  "sigma"):
            setattr(s, k, _addr(getattr(self, k)).value)
        s.nbr_offsets = _addr(self.offsets).value
        s.nbr_idx = _addr(self.idx).value
        s.N = _addr(self.N).value
        s.dN = _addr(self.dN).value
        s.xp_prev = _addr(self.xp_prev).value if self.stab else None
        s.dFm1 = _addr(self.dFm1).value if self.stab else None
        s.failed = _addr(self.failed).value if self.fracture else None
        s.tool_gt = _addr(self.tool_gt).value if self.tool else None
        s.clock = _addr(self.clock).value if self.tool else None
        s.heat = _addr(self.heat).value if self.cond else None
        s.qflux = _addr(self.qflux).value if self.cond else None
        s.node_capacity = self.ncap

    # ---------------------------------------------------------------- calls
    def init(self):
        check(lib().otm_init(C.byref(self.st), C.byref(self.p), self.dt, _ptr(self.v0), self.mode,
                             self.ws.ptr, self.ws.nbytes, _ptr(self.diag), _stream()), "otm_init")
        self.n = 0
        return self

    def step(self, rebuild=True):
        check(lib().otm_step(C.byref(self.st), C.byref(self.p), self.dt, 1 if rebuild else 0,
                             self.mode, self.ws.ptr, self.ws.nbytes, _ptr(self.diag), _stream()),
              "otm_step")
        self.n += 1

    def step_into(self, lists, rebuild=True):
        """One step whose new support lists and shape functions go to the
        tensors of ``lists`` (a dict with offsets, idx, N, dN shaped like this
        Sim's); afterwards the Sim uses those tensors, and the ones it used
        before still hold the previous step's lists, unchanged."""
        out = _lib.Lists()
        out.nbr_offsets = _ptr(lists["offsets"]).value
        out.nbr_idx = _ptr(lists["idx"]).value
        out.N = _ptr(lists["N"]).value
        out.dN = _ptr(lists["dN"]).value
        check(lib().otm_step_into(C.byref(self.st), C.byref(out), C.byref(self.p), self.dt,
                                  1 if rebuild else 0, self.mode, self.ws.ptr, self.ws.nbytes,
                                  _ptr(self.diag), _stream()), "otm_step_into")
        self.offsets, self.idx, self.N, self.dN = (lists["offsets"], lists["idx"], lists["N"],
                                                   lists["dN"])
        self.n += 1

    def use_lists(self, lists):
        """Point the state at other list / shape-function tensors (no copy).
        Graphs captured before keep the old addresses."""
        for k in ("offsets", "idx", "N", "dN"):
            t = lists[k]
            ref = getattr(self, k)
            if t.shape != ref.shape or t.dtype != ref.dtype or t.device != ref.device:
                raise ValueError(f"lists[{k!r}] does not match the state's {k}")
        self.offsets, self.idx, self.N, self.dN = (lists["offsets"], lists["idx"], lists["N"],
                                                   lists["dN"])
        self._fill_state()
        self.layout += 1

    def run(self, steps, rebuild_every=1):
        for _ in range(steps):
            self.step(rebuild=((self.n + 1) % rebuild_every == 0))

    def capture(self, steps=1, rebuild=True):
        """A HIP graph of ``steps`` consecutive otm_step calls on this state
        (lists rebuilt every step if ``rebuild``).  One replay advances the
        state by ``steps`` steps with a single launch, which pays off when a
        step is short enough for kernel launches to dominate.  The graph holds
        this Sim's device pointers, sizes and component strides: it is valid
        until ``erode`` (which shrinks the MP arrays) or ``use_lists`` (which
        points the state at other arrays), after which replaying it raises
        and the steps must be captured again.  The step path records no
        memset and no host synchronisation.  Take at least one eager step
        first, so that every kernel is loaded before capture."""
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize(self.device)
        with torch.cuda.graph(g):
            for _ in range(steps):
                check(lib().otm_step(C.byref(self.st), C.byref(self.p), self.dt,
                                     1 if rebuild else 0, self.mode, self.ws.ptr, self.ws.nbytes,
                                     _ptr(self.diag), _stream()), "otm_step (capture)")
        return StepGraph(self, g, steps)

    def refresh(self, rebuild=True):
        check(lib().otm_refresh(C.byref(self.st), C.byref(self.p), 1 if rebuild else 0, self.mode,
                                self.ws.ptr, self.ws.nbytes, _ptr(self.diag), _stream()),
              "otm_refresh")

    def erode(self):
        """Remove the failed MPs from the body (otm_erode) and recompute the
        lists, shape functions, mass and force of the rest; with
        ``insert_dist`` nodes are first added at the freed surface and with
        ``delete_orphans`` the nodes left in no support are removed.  The
        per-MP and node tensors become views of their first n entries per
        component (the memory stays allocated).  Returns the number of MPs
        removed; ``node_events`` holds (nodes added, nodes deleted)."""
        removed = C.c_int64(0)
        events = (C.c_int64 * 2)()
        check(lib().otm_erode(C.byref(self.st), C.byref(self.p), self.mode, self.ws.ptr,
                              self.ws.nbytes, _ptr(self.diag), C.byref(removed), events,
                              _stream()), "otm_erode")
        n = int(self.st.n_mp)
        for k in ("xp", "lam", "Fd", "bed", "sigma") + (("qflux",) if self.cond else ()):
            t = getattr(self, k)
            setattr(self, k, t.reshape(-1)[: t.shape[0] * n].view(t.shape[0], n))
        for k in ("vol", "mass", "epsbar", "T", "failed"):
            setattr(self, k, getattr(self, k)[:n])
        self.offsets = self.offsets[: n + 1]
        self.n_mp = n
        nn = int(self.st.n_nodes)
        for k in self._node_bufs:
            setattr(self, k, self._node_view(k, nn))
        self.n_nodes = nn
        self.node_events = (int(events[0]), int(events[1]))
        self._fill_state()
        self.layout += 1
        return int(removed.value)

    # ------------------------------------------------------- save / resume
    _SAVED = ("x", "du", "m", "f", "xp", "vol", "mass", "lam", "Fd", "bed", "epsbar", "T",
              "sigma", "offsets", "idx", "N", "dN", "xp_prev", "dFm1", "failed", "tool_gt",
              "clock", "v0", "heat", "qflux")

    def state_dict(self):
        """Host copies of every state array and the step count: what a later
        ``load_state_dict`` (on a Sim of the same workload, parameters,
        precision and pair capacity) needs to resume the run exactly."""
        torch.cuda.synchronize(self.device)
        d = {k: getattr(self, k).detach().cpu().clone() for k in self._SAVED
             if getattr(self, k) is not None}
        d["n"] = int(self.n)
        return d

    def load_state_dict(self, d):
        """Resume from ``state_dict()``.  Every saved array is put back, the
        saved support lists included (with a list skin they are not what a
        search at the saved positions would give); a refresh without a search
        then rebuilds what the workspace derives from those lists (the
        segmented mode's influence lists), and the saved arrays it recomputed
        (shape functions, multipliers, mass, force) are put back again."""
        for k in self._SAVED:
            t = getattr(self, k)
            if t is None:
                continue
            if k not in d or tuple(d[k].shape) != tuple(t.shape) or d[k].dtype != t.dtype:
                raise ValueError(f"saved {k!r} does not match this simulation")
        for k in self._SAVED:
            if getattr(self, k) is not None:
                getattr(self, k).copy_(d[k])
        self.refresh(rebuild=False)
        for k in self._SAVED:
            if getattr(self, k) is not None:
                getattr(self, k).copy_(d[k])
        self.n = int(d["n"])
        return self

    def save(self, path):
        torch.save(self.state_dict(), path)

    def load(self, path):
        return self.load_state_dict(torch.load(path, weights_only=True))

    def check_diag(self, raise_on_error=True):
        code, d = read_diag(self.diag)
        if raise_on_error and code != _lib.OTM_OK:
            raise _lib.OtmError(code, f"device diagnostics (pairs needed {d.pairs_needed}, "
                                      f"capacity {self.cap})")
        return code, d

    # ---------------------------------------------------------------- read back
    def fields(self):
        """Host copies in plain layouts: vectors (n,3), tensors (n,3,3)."""
        torch.cuda.synchronize(self.device)
        g = lambda t: t.detach().double().cpu().numpy()
        out = dict(x=g(self.x).T.copy(), du=g(self.du).T.copy(), m=g(self.m), f=g(self.f).T.copy(),
                   xp=g(self.xp).T.copy(), vol=g(self.vol), lam=g(self.lam).T.copy(),
                   epsbar=g(self.epsbar), T=g(self.T))
        Fd = g(self.Fd).T.reshape(-1, 3, 3)
        out["F"] = Fd + np.eye(3)
        out["Fd"] = Fd
        for name in ("bed", "sigma"):
            v = g(getattr(self, name)).T
            M = np.zeros((v.shape[0], 3, 3))
            for c, (i, j) in enumerate(SYM):
                M[:, i, j] = v[:, c]
                M[:, j, i] = v[:, c]
            out[name] = M
        out["be"] = out["bed"] + np.eye(3)
        off = self.offsets.cpu().numpy()
        P = int(off[-1])
        out["offsets"] = off
        out["idx"] = self.idx[:P].cpu().numpy()
        out["N"] = g(self.N[:P])
        out["dN"] = g(self.dN[:, :P]).T.copy()
        if self.fracture:
            out["failed"] = self.failed.cpu().numpy().astype(bool)
        if self.tool:
            out["gT"] = g(self.tool_gt).T.copy()
            out["clock"] = float(self.clock.cpu()[0])
        if self.cond:
            out["q"] = g(self.qflux).T.copy()
            out["heat_h"], out["heat_Q"] = g(self.heat)
        return out


class StepGraph:
    """Replayable capture of a fixed number of steps of one Sim, valid while
    the Sim's array layout is the one it was captured with."""

    def __init__(self, sim, graph, steps):
        self.sim, self.graph, self.steps = sim, graph, steps
        self.layout = sim.layout

    def replay(self):
        if self.sim.layout != self.layout:
            raise RuntimeError("the simulation's arrays changed since this graph was captured "
                               "(erosion or swapped lists): capture the steps again")
        self.graph.replay()
        self.sim.n += self.steps
