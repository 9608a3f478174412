#!/usr/bin/env python3
"""Material-point steps per second of the explicit OTM step on one MI355X.

Workload: the Taylor-rod-shaped cylinder (R = 3.2 mm, L = 21.12 mm,
h = 0.15033 mm: 202,053 nodes, 1,132,320 tet-centroid MPs), J2 plasticity
with Johnson-Cook hardening and adiabatic heating, rigid wall, support
lists rebuilt every step.  A step is one full pass of the hot path: node
update, MP update (kinematics + return map), linked-cell search, LME shape
functions and nodal force assembly.

The main line is float64 with atomic assembly; the two mixed-precision modes
(float32 return map and force products; float32 storage with float64
arithmetic) and the deterministic (segmented) assembly are timed the same way
and reported under "variants", as is the step with the stabilisation term
(eps = mu h^2), together with the Taylor rod and the chip-formation workpiece
at the paper's own sizes (27,840 and 108,000 MPs, 2000 steps each; eager and
graph-replayed) beside the paper's per-step times, and the 6.1M-MP cutting
workload with erosion and heat conduction.  Inputs are resident in HBM before the timed region; the
timed region is bracketed by device synchronisation and HIP events on the
stream the kernels run on.  Per-phase durations come from events recorded by
the library between its kernels (otm_step_profiled).

    python bench.py [--gpus 1] [--steps 100] [--warmup 5]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
PHASES = ("node_update", "mp_update", "search", "lme", "assembly", "segmented", "end")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_mp_update_taylor_rod.txt")


# ------------------------------------------------------- algorithmic bytes
def mp_pass_bytes(n_mp, n_nodes, P, precision, model, conduction=False):
    """Minimum HBM bytes of one MP-pass launch (each array read or written
    once).  Per pair: idx 4 + N 8 + grad N 24 (12 in mixed).  Per MP: read
    offsets 8, vol 8, F-1 72 (36), b^e-1 48 (24), epsbar 8, T 8; write x_p 24,
    vol 8, F-1, b^e-1, epsbar, T, sigma 48 (24).  Per node: x and du gathered
    once, 48.  With conduction: per node the temperature and its rate, 16;
    per MP the heat flux written, 24."""
    r = 8 if precision == "fp64" else 4
    pair = 4 + 8 + 3 * r
    plastic = model != 0
    read = 8 + 8 + 9 * r + (6 * r + 8 + 8 if plastic else 0)
    write = 24 + 8 + 9 * r + 6 * r + (6 * r + 8 + 8 if plastic else 0)
    if conduction:
        write += 24
    return pair * P + (read + write) * n_mp + (64 if conduction else 48) * n_nodes


def lme_bytes(n_mp, n_nodes, P, precision):
    """Shape functions: per pair idx 4 read, N 8 and grad N 24 (12) written;
    per MP offsets 8, x_p 24 and lambda 24 read, lambda 24 written; per node
    x 24 gathered once."""
    r = 8 if precision == "fp64" else 4
    return (4 + 8 + 3 * r) * P + 80 * n_mp + 24 * n_nodes


def lme_assembly_bytes(n_mp, n_nodes, P, precision):
    """Shape functions with the atomic assembly fused in (one kernel): the
    LME traffic plus, per MP, vol, mass and sigma read and, per node, m and f
    read-modify-written; the pairs' N and grad N are assembled from registers
    and not read back."""
    r = 8 if precision == "fp64" else 4
    return lme_bytes(n_mp, n_nodes, P, precision) + (16 + 6 * r) * n_mp + 64 * n_nodes


def search_bytes(n_mp, n_nodes, P):
    """Count and fill passes: x_p read twice (48), offsets written and read
    (16), idx written (4 per pair); nodes binned once (x read 24, cell id
    written and read 8, sorted copy written 32, read back by both passes
    from cache at least once 32)."""
    return 4 * P + 64 * n_mp + 96 * n_nodes


def node_bytes(n_nodes):
    return 160 * n_nodes


def src_digest():
    """Digest of the sources the MP-pass kernel is compiled from."""
    h = hashlib.sha256()
    for f in ("mp_update.hip", "constitutive.h", "otm_common.h", "launch.h"):
        h.update(open(os.path.join(ROOT, "paper_2206_08772_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per MP-pass launch from committed rocprofv3 counters, or
    None if there are none or the kernel source changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m = re.search(r"^source_digest:\s*(\S+)", txt, re.M)
    b = re.search(r"^hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt, re.M)
    if not m or not b or m.group(1) != src_digest():
        return None
    return float(b.group(1))


# ------------------------------------------------------------ GPU timing
def hip_runtime():
    """The HIP runtime already loaded by torch (events are created with it)."""
    import ctypes as C
    for name in ("libamdhip64.so", "libamdhip64.so.7", "libamdhip64.so.6"):
        try:
            rt = C.CDLL(name)
            break
        except OSError:
            continue
    else:
        raise OSError("libamdhip64 not found")
    rt.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
    rt.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
    rt.hipEventDestroy.argtypes = [C.c_void_p]
    return rt


def run_variant(w, precision, scatter, steps, warmup, **over):
    import ctypes as C
    import torch
    import otm_workloads as W
    from paper_2206_08772_amd import _lib
    from paper_2206_08772_amd.sim import Sim, _ptr, _stream

    p = W.params_from_workload(w, **over)
    sim = Sim(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, precision=precision,
              scatter=scatter)
    sim.init()
    for _ in range(warmup):
        sim.step()
    sim.check_diag()
    torch.cuda.synchronize()
    lib = _lib.lib()
    rt = hip_runtime()
    skip = ("segmented",) if scatter == "atomic" else ()
    arrays = []
    for _ in range(steps):
        a = (C.c_void_p * len(PHASES))()
        for k, name in enumerate(PHASES):
            if name in skip:
                a[k] = None
            else:
                ev = C.c_void_p()
                assert rt.hipEventCreate(C.byref(ev)) == 0
                a[k] = ev
        arrays.append(a)
    stream = _stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for k in range(steps):
        _lib.check(lib.otm_step_profiled(C.byref(sim.st), C.byref(sim.p), sim.dt, 1, sim.mode,
                                         sim.ws.ptr, sim.ws.nbytes, _ptr(sim.diag), arrays[k],
                                         stream), "otm_step_profiled")
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    code, d = sim.check_diag()
    used = [k for k in range(len(PHASES)) if PHASES[k] not in skip]
    phase_ms = {}
    ms = C.c_float()
    for a, b in zip(used[:-1], used[1:]):
        acc = 0.0
        for s in range(steps):
            assert rt.hipEventElapsedTime(C.byref(ms), arrays[s][a], arrays[s][b]) == 0
            acc += ms.value
        phase_ms[PHASES[a]] = acc / steps
    for a in arrays:
        for k in used:
            rt.hipEventDestroy(a[k])
    P = int(d.pairs_needed)
    out = dict(ms_per_step=total_ms / steps, wall_s=wall, value=w.n_mp * steps / (total_ms / 1e3),
               phase_ms=phase_ms, pairs=P, kbar=P / w.n_mp, max_support=int(d.max_support))
    del sim
    torch.cuda.empty_cache()
    return out


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Best of ``reps`` device-to-device copies of ``nbytes`` (one copy kernel
    each, timed with events): bytes read plus written over its time, GB/s.  A
    measured ceiling for streaming kernels, beside the vendor peak."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (best * 1e-3) / 1e9


def roofline_entry(nbytes, ms):
    gbs = nbytes / (ms * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 4))


# ------------------------------------------------- the paper's own rod size
# The paper's Taylor-rod timing table (Sec. 4.1): 2000 steps of 28,423 MPs on
# Haswell cores, total wall time 2697.26 s on 1 core and 23.78 s on 239 cores
# (whole parallel step, halo exchange and VTK output included).
PAPER_ROD_S_PER_STEP = {"1_core": 2697.26 / 2000, "239_cores": 23.78 / 2000}
PAPER_CHIP_S_PER_STEP = {"1_core": 11348.8932 / 2000, "549_cores": 33.589 / 2000}


def run_paper_rod(warmup=5, graph_steps=10):
    """The Taylor rod of Sec. 4.1 at the paper's size (5,959 nodes, 27,840
    MPs, linear hardening, 227 m/s, dt = 4e-9 s), float64 with atomic
    assembly and lists rebuilt every step, timed over all 2000 steps of the
    paper's run: eager otm_step calls, and replays of a HIP graph of
    ``graph_steps`` captured steps (one launch per replay)."""
    import otm_workloads as W
    w = W.config_by_name("paper_rod")
    out = _run_paper_size(w, f"{w.name}: {w.n_nodes} nodes, {w.n_mp} MPs, J2 linear hardening, "
                             f"dt 4e-9 s, {w.steps} steps, float64, atomic assembly",
                          PAPER_ROD_S_PER_STEP, warmup, graph_steps)
    out["note"] = ("paper: 28,423 MPs on Haswell cores, whole parallel step including halo "
                   "exchange and output; context, not a target")
    return out


def run_cutting(warmup=5, graph_steps=10):
    """The chip-formation workpiece of Sec. 4.2 at the paper's size (27,633
    nodes, 108,000 MPs; JC flow and fracture, tool contact with Coulomb
    friction, dt = 1e-10 s), float64 with atomic assembly, all 2000 steps,
    eager and graph-replayed; reports the failed MPs and nodes in contact at
    the end of the eager run."""
    import otm_workloads as W
    w = W.config_by_name("cutting_slab")
    out = _run_paper_size(w, f"{w.name}: {w.n_nodes} nodes, {w.n_mp} MPs, JC flow + fracture, "
                             f"tool at {-w.tool['v'][0]:g} m/s with Coulomb friction "
                             f"{w.tool['mu']}, dt 1e-10 s, {w.steps} steps, float64, "
                             "atomic assembly", PAPER_CHIP_S_PER_STEP, warmup, graph_steps)
    out["note"] = ("paper: 27,417 nodes / 107,975 MPs on Haswell cores, whole parallel step "
                   "including halo exchange and output; context, not a target")
    return out


def _run_paper_size(w, label, paper_s, warmup, graph_steps):
    import torch
    import otm_workloads as W
    from paper_2206_08772_amd.sim import Sim
    p = W.params_from_workload(w)
    steps = w.steps
    out = dict(workload=label, steps=steps)
    for mode in ("eager", "graph"):
        sim = Sim(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, precision="fp64")
        sim.init()
        for _ in range(warmup):
            sim.step()
        g = sim.capture(graph_steps) if mode == "graph" else None
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        if g is None:
            for _ in range(steps):
                sim.step()
        else:
            for _ in range(steps // graph_steps):
                g.replay()
        t1.record()
        torch.cuda.synchronize()
        sim.check_diag()
        ms = t0.elapsed_time(t1) / steps
        out[mode] = dict(ms_per_step=round(ms, 4), value=round(w.n_mp / (ms * 1e-3), 1))
        if mode == "eager" and sim.fracture:
            out["failed_mps_at_end"] = int(sim.failed.sum())
        if mode == "eager" and sim.tool:
            out["nodes_with_tangential_gap_at_end"] = int((sim.tool_gt.abs().sum(0) > 0).sum())
        if mode == "eager" and sim.fracture:
            # removal of the failed MPs and the refresh of the rest, host wall time
            torch.cuda.synchronize()
            t = time.perf_counter()
            removed = sim.erode()
            torch.cuda.synchronize()
            sim.check_diag()
            out["erode"] = dict(removed=removed, n_mp_after=sim.n_mp,
                                ms=round(1e3 * (time.perf_counter() - t), 3))
        del sim, g
        torch.cuda.empty_cache()
    best = min(out["eager"]["ms_per_step"], out["graph"]["ms_per_step"]) * 1e-3
    out["paper_s_per_step"] = {k: round(v, 5) for k, v in paper_s.items()}
    out["speedup_vs_paper"] = {k: round(v / best, 1) for k, v in paper_s.items()}
    return out


def run_cutting_5m(erode_every=50):
    """Orthogonal cutting at production scale (cutting_slab_5m: 2 x 1 x
    0.05 mm, ~1.1M nodes, ~6.1M MPs): mixed precision, atomic assembly,
    lists rebuilt every step, JC flow and fracture, tool contact, heat
    conduction, and every ``erode_every`` steps the failed MPs removed with
    nodes added at the freed surface and orphan nodes deleted.  Steps are
    timed with HIP events (per phase through otm_step_profiled); each
    erosion (which synchronises) is timed on the host."""
    import ctypes as C
    import torch
    import otm_workloads as W
    from paper_2206_08772_amd import _lib
    from paper_2206_08772_amd.sim import Sim, _ptr, _stream
    w = W.config_by_name("cutting_slab_5m")
    p = W.params_from_workload(w)
    # kernels of these switches loaded on the small cut first
    ws_ = W.config_by_name("small_cut")
    warm = Sim(ws_.x_nodes, ws_.x_mp, ws_.vol_mp, ws_.mass_mp, ws_.v0_nodes,
               W.params_from_workload(ws_, kappa=p["kappa"], insert_dist=0.5 * ws_.h,
                                      delete_orphans=True), precision="mixed")
    warm.init()
    warm.run(3)
    warm.erode()
    warm.check_diag()
    del warm
    sim = Sim(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, precision="mixed")
    sim.init()
    sim.check_diag()
    lib = _lib.lib()
    rt = hip_runtime()
    stream = _stream()
    steps = w.steps
    used = [k for k, n in enumerate(PHASES) if n != "segmented"]
    ev = []
    for _ in range(steps):
        a = (C.c_void_p * len(PHASES))()
        for k in used:
            e = C.c_void_p()
            assert rt.hipEventCreate(C.byref(e)) == 0
            a[k] = e
        ev.append(a)
    ms = C.c_float()
    step_ms, mp_ms, mp_bytes, mp_steps = 0.0, 0.0, 0.0, 0
    phase_acc = {PHASES[k]: 0.0 for k in used[:-1]}
    erode_ms, removed, inserted, deleted = [], 0, 0, 0
    torch.cuda.synchronize()
    for s0 in range(0, steps, erode_every):
        n_seg = min(erode_every, steps - s0)
        n_mp, n_nodes = sim.n_mp, sim.n_nodes
        for k in range(s0, s0 + n_seg):
            _lib.check(lib.otm_step_profiled(C.byref(sim.st), C.byref(sim.p), sim.dt, 1, sim.mode,
                                             sim.ws.ptr, sim.ws.nbytes, _ptr(sim.diag), ev[k],
                                             stream), "otm_step_profiled")
        torch.cuda.synchronize()
        try:
            code, d = sim.check_diag()
        except _lib.OtmError as e:
            raise RuntimeError(f"steps {s0 + 1}..{s0 + n_seg} after {len(erode_ms)} "
                               f"erosions: {e}") from None
        P = int(d.pairs_needed)
        for k in range(s0, s0 + n_seg):
            for a, b in zip(used[:-1], used[1:]):
                assert rt.hipEventElapsedTime(C.byref(ms), ev[k][a], ev[k][b]) == 0
                phase_acc[PHASES[a]] += ms.value
                step_ms += ms.value
                if PHASES[a] == "mp_update":
                    mp_ms += ms.value
        mp_bytes += n_seg * mp_pass_bytes(n_mp, n_nodes, P, "mixed", w.material.model, True)
        mp_steps += n_seg * n_mp
        t = time.perf_counter()
        removed += sim.erode()
        torch.cuda.synchronize()
        erode_ms.append(1e3 * (time.perf_counter() - t))
        inserted += sim.node_events[0]
        deleted += sim.node_events[1]
        sim.check_diag()
    for a in ev:
        for k in used:
            rt.hipEventDestroy(a[k])
    out = dict(
        workload=f"{w.name}: 2 x 1 x 0.05 mm slab, {w.n_nodes} nodes, {w.n_mp} MPs, JC flow + "
                 f"fracture, tool at 5 m/s, heat conduction (kappa {p['kappa']} W/(m K)), "
                 f"rebuild every step, mixed precision, atomic assembly, erosion every "
                 f"{erode_every} steps with nodes added at the freed surface and orphans "
                 f"deleted, {steps} steps",
        steps=steps, ms_per_step=round(step_ms / steps, 4),
        value=round(mp_steps / (step_ms * 1e-3), 1), unit="material-point steps/s",
        phase_ms={k: round(v / steps, 4) for k, v in phase_acc.items()},
        mp_pass_roofline=roofline_entry(mp_bytes / steps, mp_ms / steps),
        erosion=dict(calls=len(erode_ms), removed_mps=removed, nodes_added=inserted,
                     nodes_deleted=deleted, ms_mean=round(sum(erode_ms) / len(erode_ms), 2)),
        n_mp_at_end=sim.n_mp, n_nodes_at_end=sim.n_nodes,
        max_temperature_rise=round(float((sim.T - p["T_r"]).max()), 3))
    del sim
    torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------ adjoint ratio
def adjoint_ratio(every=20):
    """Gradient of a rollout loss on the adjoint-rod workload (268k MPs, 200
    float64 steps): wall time of the backward sweep (segment replay from
    checkpoints every ``every`` steps + otm_step_adjoint) over the wall time
    of the plain forward rollout of the same steps."""
    import torch
    import otm_workloads as W
    from paper_2206_08772_amd.adjoint import AdjointBuffers, rollout_backward, rollout_forward
    from paper_2206_08772_amd.sim import Sim
    w = W.config_by_name("adjoint_rod")
    p = W.params_from_workload(w)
    steps = w.steps
    sim = Sim(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    sim.init()
    sim.run(3)                          # warm-up (kernels loaded, caches)
    sim.init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    target = sim.x.clone() * (1.0 + 1e-6)
    # the sweep's buffers (tape, adjoints, workspace) are set up before the
    # timed region, as the forward's state is, and one segment of the sweep
    # runs first, as the forward's warm-up steps do (first launches load the
    # adjoint kernels)
    bufs = AdjointBuffers(sim, every, steps)
    sim.init()
    ck_w = rollout_forward(sim, every, every)
    rollout_backward(sim, ck_w, every, every, sim.x - target, bufs=bufs)
    sim.init()
    ckpt = rollout_forward(sim, steps, every)
    xbar = sim.x - target
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta_bar, _ = rollout_backward(sim, ckpt, steps, every, xbar, bufs=bufs)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    return dict(ratio=round(t_bwd / t_fwd, 3), forward_s=round(t_fwd, 4),
                backward_s=round(t_bwd, 4), workload=f"{w.name}: {w.n_mp} MPs, {steps} steps, "
                f"checkpoint every {every}", theta_bar_finite=bool(torch.isfinite(theta_bar).all()))


# ------------------------------------------------------------ CPU baseline
def cpu_baseline(seconds_budget=30.0):
    """The oracle, as it is, on a bounded slab of the same rod (same h,
    radius, material and seed; 12 lattice layers instead of 141), single
    thread, timing steps after its t = 0 set-up."""
    from threadpoolctl import threadpool_limits
    import otm_workloads as W
    from oracle import step as OST
    h = 0.15033e-3
    w = W.taylor_rod(h=h, seed=1, length=12.5 * h, name="taylor_rod_slab")
    p = W.params_from_workload(w)
    with threadpool_limits(limits=1):
        st = OST.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
        t0 = time.perf_counter()
        n = 0
        while True:
            OST.step(st, p)
            n += 1
            if time.perf_counter() - t0 > seconds_budget / 3 or n >= 10:
                break
        dt = time.perf_counter() - t0
    return dict(value=round(w.n_mp * n / dt, 1), unit="material-point steps/s", cores=1,
                kind="oracle",
                sample=f"NumPy oracle, 1 thread: {n} steps of a {w.n_mp}-MP, {w.n_nodes}-node "
                       f"slab (12 lattice layers) of the same rod after its t=0 set-up; "
                       f"{dt:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="taylor_rod")
    ap.add_argument("--variants",
                    default="mixed,mixed_storage,segmented,stabilised,paper_rod,cutting,"
                            "cutting_5m",
                    help="extra timed variants: mixed, mixed_storage, segmented, stabilised, "
                         "paper_rod, cutting, cutting_5m (comma separated, or none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="print only the adjoint/forward time ratio (one JSON line)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (a reference kernel "
                         "of known traffic for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import otm_workloads as W
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))
    if args.calibration_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.adjoint_only:
        print(json.dumps(adjoint_ratio()), flush=True)
        return
    w = W.config_by_name(args.workload)

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    progress(f"main line: {w.name}, fp64, atomic, {args.steps} steps")
    main_run = run_variant(w, "fp64", "atomic", args.steps, args.warmup)
    copy_gbs = copy_bandwidth()
    variants = {}
    for v in [s for s in args.variants.split(",") if s and s != "none"]:
        progress(f"variant {v}")
        if v in ("paper_rod", "cutting", "cutting_5m"):
            run = {"paper_rod": run_paper_rod, "cutting": run_cutting,
                   "cutting_5m": run_cutting_5m}[v]
            try:
                variants[v] = run()
            except Exception as e:          # a failed variant is reported, not fatal
                variants[v] = {"error": f"{type(e).__name__}: {e}"}
                torch.cuda.synchronize()
                torch.cuda.empty_cache()
            continue
        prec = v if v in ("mixed", "mixed_storage") else "fp64"
        scat = "segmented" if v == "segmented" else "atomic"
        over = {}
        if v == "stabilised":       # the stabilisation term with eps = mu h^2
            over["eps_stab"] = w.material.E / (2 * (1 + w.material.nu)) * w.h ** 2
        r = run_variant(w, prec, scat, args.steps, args.warmup, **over)
        pm = dict(r["phase_ms"])
        if scat == "segmented":      # markers 3..6: lists, LME + contributions, node sums
            pm["influence_lists"] = pm.pop("lme")
            pm["lme_contributions"] = pm.pop("assembly")
            pm["node_sums"] = pm.pop("segmented")
        elif not over:               # assembly fused into the shape-function kernel
            pm["lme_assembly"] = pm.pop("lme") + pm.pop("assembly")
        variants[v] = dict(value=round(r["value"], 1), ms_per_step=round(r["ms_per_step"], 4),
                           phase_ms={k: round(x, 4) for k, x in pm.items()})
        if over:
            variants[v]["eps_stab"] = over["eps_stab"]
        if prec != "fp64":
            nb = mp_pass_bytes(w.n_mp, w.n_nodes, r["pairs"], "mixed", w.material.model)
            variants[v]["mp_pass_roofline"] = roofline_entry(nb, r["phase_ms"]["mp_update"])

    P = main_run["pairs"]
    ph = main_run["phase_ms"]
    mp_b = mp_pass_bytes(w.n_mp, w.n_nodes, P, "fp64", w.material.model)
    roof = roofline_entry(mp_b, ph["mp_update"])
    roof["kernel"] = "k_mp_update<double> (MP pass: kinematics + J2/JC return map)"
    roof["traffic"] = measured_traffic()
    # the same kernel against a measured 1 GiB device-to-device copy
    roof["measured_copy_gbs"] = round(copy_gbs, 1)
    roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)
    phases = {
        "node_update": roofline_entry(node_bytes(w.n_nodes), ph["node_update"]),
        "search": roofline_entry(search_bytes(w.n_mp, w.n_nodes, P), ph["search"]),
        # the atomic assembly runs inside the shape-function kernel: one phase
        "lme_assembly": roofline_entry(lme_assembly_bytes(w.n_mp, w.n_nodes, P, "fp64"),
                                       ph["lme"] + ph["assembly"]),
    }
    for k in phases:
        phases[k]["ms"] = round(ph["lme"] + ph["assembly"] if k == "lme_assembly" else ph[k], 4)
    phases["mp_update"] = dict(roof, ms=round(ph["mp_update"], 4))
    # `roofline` is the MP pass (the kernel the HBM target is set on); the
    # longest kernel is the shape functions with the fused assembly
    longest = dict(kernel="k_lme_asm<double> (LME Newton + fused atomic assembly)",
                   ms=phases["lme_assembly"]["ms"],
                   share_of_step=round(phases["lme_assembly"]["ms"] / main_run["ms_per_step"], 3),
                   hbm_frac=phases["lme_assembly"]["frac"],
                   bound="latency of the per-MP Newton chain at two waves per SIMD; FP64 VALU "
                         "issue ~15 % of peak (profiles/valu_taylor_rod_fp64_mixed.md)")

    line = {
        "metric": "material-point steps/s (FP64 vs mixed, 1 GPU) + adjoint/forward time ratio",
        "value": round(main_run["value"], 1),
        "unit": "material-point steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: J2/Johnson-Cook "
                               f"{'workpiece with fracture and tool contact' if w.tool else 'rod'}, "
                               f"{w.n_nodes} nodes, {w.n_mp} MPs, rebuild every step, "
                               "atomic assembly",
                   "n_nodes": w.n_nodes, "n_mp": w.n_mp, "pairs": P,
                   "mean_support": round(main_run["kbar"], 3),
                   "max_support": main_run["max_support"], "parallelism": "single GPU"},
        "roofline": roof,
        "longest_kernel": longest,
        "phases": phases,
        "variants": variants,
        "adjoint_forward_ratio": None,
    }
    if not args.no_adjoint:
        progress("adjoint rollout")
        adj = adjoint_ratio()
        line["adjoint_forward_ratio"] = adj["ratio"]
        line["adjoint"] = adj
    if not args.no_cpu_baseline:
        progress("oracle on the host")
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
