"""Parity of the HIP path (through the C ABI) with the CPU oracle."""
import json
import os

import numpy as np
import pytest

import otm_workloads as W
from oracle import lme as OL
from oracle import search as OS
from oracle import step as OST
from tests.gpu_common import make_sim, require_gpu, to_dev
from tests.helpers import compare, gpu_fields, oracle_fields, rel_err

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "search_tiny.json")
FP64_TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _gpu_lists(X, P, r, cell=None, cap=None):
    from paper_2206_08772_amd.sim import build_neighbors
    off, idx = build_neighbors(to_dev(X), to_dev(P), r, cell or r * 1.0001, cap)
    return off.cpu().numpy(), idx.cpu().numpy()


# ------------------------------------------------------------------ search
def test_search_golden_inclusive_boundary():
    g = json.load(open(GOLDEN))
    off, idx = _gpu_lists(np.array(g["nodes"], float), np.array(g["mps"], float), g["radius"],
                          g["radius"])
    rows = [list(idx[off[i]:off[i + 1]]) for i in range(len(off) - 1)]
    assert rows == g["expected"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_search_bitexact_random(seed):
    X, P = W.random_cloud(3000, 2500, seed)
    P[:100] = P[:100] * 1.5 - 0.25      # MPs outside the node box
    for r in (0.05, 0.11):
        o_ref, i_ref = OS.neighbors_bruteforce(X, P, r)
        o, i = _gpu_lists(X, P, r)
        assert np.array_equal(o, o_ref)
        assert np.array_equal(i, i_ref)


def test_search_bitexact_workloads(cube):
    for w in (cube, W.config_by_name("small_rod")):
        o_ref, i_ref = OS.neighbors_bruteforce(w.x_nodes, w.x_mp, w.r_list)
        o, i = _gpu_lists(w.x_nodes, w.x_mp, w.r_list)
        assert np.array_equal(o, o_ref) and np.array_equal(i, i_ref)


def test_search_long_supports_and_lattice_ties():
    """Supports longer than the LDS sort buffer (64) and distances that tie
    the radius exactly on an unjittered lattice."""
    g = np.arange(0, 12) * 0.5
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    P = X[::7] + np.array([0.0, 0.0, 0.0])
    for r in (1.0, 1.5, 2.0):          # r^2 hits lattice distances exactly
        o_ref, i_ref = OS.neighbors_bruteforce(X, P, r)
        o, i = _gpu_lists(X, P, r)
        assert np.diff(o_ref).max() > 64 or r < 1.5
        assert np.array_equal(o, o_ref) and np.array_equal(i, i_ref)


def test_search_capacity_error_reports_count():
    import ctypes as C
    import torch
    from paper_2206_08772_amd import _lib
    from paper_2206_08772_amd.sim import Workspace, _ptr, _stream
    X, P = W.random_cloud(500, 400, 4)
    o_ref, _ = OS.neighbors_bruteforce(X, P, 0.2)
    need = int(o_ref[-1])
    xn, xm = to_dev(X), to_dev(P)
    off = torch.empty(401, dtype=torch.int64, device="cuda")
    idx = torch.full((need // 2,), -7, dtype=torch.int32, device="cuda")
    ws = Workspace(500, 400, need // 2, "cuda")
    n = C.c_int64(0)
    code = _lib.lib().otm_build_neighbors(500, _ptr(xn), 400, _ptr(xm), 0.2, 0.2, need // 2,
                                          _ptr(off), _ptr(idx), C.byref(n), ws.ptr, ws.nbytes,
                                          _stream())
    assert code == _lib.OTM_ERR_CAPACITY
    assert n.value == need
    assert np.all(idx.cpu().numpy() == -7)   # nothing written
    assert np.array_equal(off.cpu().numpy(), o_ref)


def test_search_empty_inputs():
    X, P = W.random_cloud(50, 40, 5)
    o, i = _gpu_lists(X, P[:0], 0.2)
    assert list(o) == [0] and i.size == 0
    o, i = _gpu_lists(X, P[:1] + 10.0, 0.2)    # an MP far from every node
    assert list(o) == [0, 0]


# ------------------------------------------------------------------ LME
def _lme_case(w, r=None, beta=None):
    r = r or w.r_list
    beta = beta or w.beta
    off, idx = OS.neighbors_bruteforce(w.x_nodes, w.x_mp, r)
    return off, idx, beta


@pytest.mark.parametrize("precision", [0, 1])
def test_lme_parity_cube(cube, precision):
    from paper_2206_08772_amd.sim import lme_shape, read_diag
    import torch
    off, idx, beta = _lme_case(cube)
    tol = 1e-13 * cube.h
    lam_ref, N_ref, dN_ref = OL.lme_shape(cube.x_nodes, cube.x_mp, off, idx, beta, tol)
    lam, N, dN, diag = lme_shape(to_dev(cube.x_nodes), to_dev(cube.x_mp),
                                 torch.from_numpy(off).cuda(), torch.from_numpy(idx).cuda(),
                                 beta, tol, precision=precision)
    assert read_diag(diag)[0] == 0
    assert rel_err(N.cpu().numpy(), N_ref) < 1e-12
    assert rel_err(lam.cpu().numpy().T, lam_ref) < 1e-9
    dn = dN.double().cpu().numpy().T
    # float32 storage of grad N in the mixed mode: one rounding
    assert rel_err(dn, dN_ref) < (1e-11 if precision == 0 else 1e-7)


def test_lme_long_supports_use_the_uncached_path():
    """gamma = 0.8 (the wide end of the paper's range): supports of ~200
    nodes, beyond the register-cached length."""
    w = W.elastic_cube(n=8)
    w.gamma = 0.8
    import torch
    from paper_2206_08772_amd.sim import lme_shape, read_diag
    off, idx = OS.neighbors_bruteforce(w.x_nodes, w.x_mp, w.r_cut)
    assert np.diff(off).max() > 64
    tol = 1e-13 * w.h
    lam_ref, N_ref, dN_ref = OL.lme_shape(w.x_nodes, w.x_mp, off, idx, w.beta, tol)
    lam, N, dN, diag = lme_shape(to_dev(w.x_nodes), to_dev(w.x_mp), torch.from_numpy(off).cuda(),
                                 torch.from_numpy(idx).cuda(), w.beta, tol)
    assert read_diag(diag)[0] == 0
    assert rel_err(N.cpu().numpy(), N_ref) < 1e-12
    assert rel_err(dN.cpu().numpy().T, dN_ref) < 1e-11


def test_lme_nonconvergence_is_reported():
    import torch
    from paper_2206_08772_amd import _lib
    from paper_2206_08772_amd.sim import lme_shape, read_diag
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0], [1, 1, 1.0]])
    P = np.array([[0.2, 0.2, 0.2], [3.0, 3.0, 3.0], [0.3, 0.1, 0.2]])
    off = np.array([0, 5, 10, 15], np.int64)
    idx = np.tile(np.arange(5, dtype=np.int32), 3)
    with pytest.raises(OL.LMENotConverged) as e:
        OL.lme_shape(X, P, off, idx, 4.0, 1e-13)
    assert e.value.mp_index == 1
    lam, N, dN, diag = lme_shape(to_dev(X), to_dev(P), torch.from_numpy(off).cuda(),
                                 torch.from_numpy(idx).cuda(), 4.0, 1e-13)
    code, d = read_diag(diag)
    assert code == _lib.OTM_ERR_LME_NOCONV
    assert d.n_lme_noconv == 1 and d.first_lme_noconv == 1


# ------------------------------------------------------------------ steps
def _oracle_run(w, steps, **over):
    p = W.params_from_workload(w, **over)
    st = OST.init_state(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p)
    for _ in range(steps):
        OST.step(st, p)
    return st, p


def _gpu_run(w, steps, precision="fp64", scatter="atomic", **over):
    sim, p = make_sim(w, precision, scatter, **over)
    sim.init()
    sim.run(steps, rebuild_every=int(p["rebuild_every"]))
    code, d = sim.check_diag()
    return sim.fields(), sim


@pytest.fixture(scope="module")
def cube_oracle(cube):
    return _oracle_run(cube, 10)


@pytest.mark.parametrize("scatter", ["atomic", "segmented"])
def test_cube_trajectory_fp64(cube, cube_oracle, scatter):
    st, p = cube_oracle
    g, _ = _gpu_run(cube, 10, scatter=scatter)
    assert np.array_equal(g["offsets"], st.offsets) and np.array_equal(g["idx"], st.idx)
    errs = compare(gpu_fields(g, cube.x_nodes, cube.x_mp, p["T_r"]),
                   oracle_fields(st, cube.x_nodes, cube.x_mp, p["T_r"]))
    bad = {k: v for k, v in errs.items() if not v < FP64_TOL}
    assert not bad, bad


@pytest.fixture(scope="module")
def rod_oracle():
    w = W.config_by_name("small_rod")
    st, p = _oracle_run(w, 100)
    return w, st, p


@pytest.mark.parametrize("scatter", ["atomic", "segmented"])
def test_small_rod_100_steps_fp64(rod_oracle, scatter):
    """J2 / Johnson-Cook with heating and the rigid wall over 100 steps."""
    w, st, p = rod_oracle
    g, _ = _gpu_run(w, 100, scatter=scatter)
    assert st.epsbar.max() > 0.05              # real plastic flow happened
    assert np.array_equal(g["offsets"], st.offsets) and np.array_equal(g["idx"], st.idx)
    errs = compare(gpu_fields(g, w.x_nodes, w.x_mp, p["T_r"]),
                   oracle_fields(st, w.x_nodes, w.x_mp, p["T_r"]))
    bad = {k: v for k, v in errs.items() if not v < FP64_TOL}
    assert not bad, bad


MIXED_TOL = {  # stated mixed-precision error bounds over 100 steps (relative, max-norm)
    "u": 1e-5, "du": 1e-5, "up": 1e-5, "vol": 1e-5, "Fm1": 1e-5, "be_m1": 1e-5,
    "sigma": 1e-5, "epsbar": 1e-5, "dT": 1e-5, "m": 1e-5, "f": 1e-5, "N": 1e-5,
    "dN": 1e-5, "lam": 1e-5,
}


@pytest.mark.parametrize("precision", ["mixed", "mixed_storage"])
def test_small_rod_100_steps_mixed(rod_oracle, precision):
    w, st, p = rod_oracle
    g, _ = _gpu_run(w, 100, precision=precision)
    assert np.array_equal(g["offsets"], st.offsets) and np.array_equal(g["idx"], st.idx)
    errs = compare(gpu_fields(g, w.x_nodes, w.x_mp, p["T_r"]),
                   oracle_fields(st, w.x_nodes, w.x_mp, p["T_r"]))
    print(f"{precision} errors after 100 steps:", json.dumps(errs))
    bad = {k: v for k, v in errs.items() if not v < MIXED_TOL[k]}
    assert not bad, bad


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_small_rod_odd_pair_capacity(rod_oracle, precision):
    """The MP update loads two consecutive pairs at once only with an even
    pair capacity (the default one is rounded up to even); an odd one takes
    the one-pair-per-load path, held to the same bounds over 100 steps."""
    from paper_2206_08772_amd.sim import Sim
    w, st, p = rod_oracle
    even, _ = make_sim(w, precision)
    assert even.cap % 2 == 0
    sim = Sim(w.x_nodes, w.x_mp, w.vol_mp, w.mass_mp, w.v0_nodes, p, precision=precision,
              pair_capacity=even.cap + 1)
    del even
    sim.init()
    sim.run(100, rebuild_every=int(p["rebuild_every"]))
    sim.check_diag()
    g = sim.fields()
    assert np.array_equal(g["offsets"], st.offsets) and np.array_equal(g["idx"], st.idx)
    errs = compare(gpu_fields(g, w.x_nodes, w.x_mp, p["T_r"]),
                   oracle_fields(st, w.x_nodes, w.x_mp, p["T_r"]))
    tol = {k: FP64_TOL for k in errs} if precision == "fp64" else MIXED_TOL
    bad = {k: v for k, v in errs.items() if not v < tol[k]}
    assert not bad, bad


def test_segmented_scatter_is_bit_reproducible():
    w = W.config_by_name("small_rod")
    a, _ = _gpu_run(w, 20, scatter="segmented")
    b, _ = _gpu_run(w, 20, scatter="segmented")
    for k in ("x", "du", "m", "f", "xp", "sigma", "N", "dN"):
        assert np.array_equal(a[k], b[k]), k
    c, _ = _gpu_run(w, 20, scatter="atomic")
    assert rel_err(c["x"] - w.x_nodes, a["x"] - w.x_nodes) < 1e-12


def test_linear_hardening_and_neo_hooke_models(cube):
    """The other two constitutive options, 10 steps each."""
    w = W.config_by_name("small_rod")
    st, p = _oracle_run(w, 10, model=W.MODEL_J2_LINEAR)
    g, _ = _gpu_run(w, 10, model=W.MODEL_J2_LINEAR)
    errs = compare(gpu_fields(g, w.x_nodes, w.x_mp, p["T_r"]),
                   oracle_fields(st, w.x_nodes, w.x_mp, p["T_r"]))
    assert st.epsbar.max() > 0
    bad = {k: v for k, v in errs.items() if not v < FP64_TOL}
    assert not bad, bad


def test_paper_rod_20_steps_fp64():
    """The Taylor rod of Sec. 4.1 at the paper's size (5,959 nodes, 27,840 MPs;
    227 m/s, linear hardening, dt = 4e-9 s): the first 20 of its 2000 steps,
    with plastic flow at the wall from the first steps."""
    w = W.config_by_name("paper_rod")
    st, p = _oracle_run(w, 20)
    g, _ = _gpu_run(w, 20)
    assert st.epsbar.max() > 0.01
    assert np.array_equal(g["offsets"], st.offsets) and np.array_equal(g["idx"], st.idx)
    errs = compare(gpu_fields(g, w.x_nodes, w.x_mp, p["T_r"]),
                   oracle_fields(st, w.x_nodes, w.x_mp, p["T_r"]))
    bad = {k: v for k, v in errs.items() if not v < FP64_TOL}
    assert not bad, bad


@pytest.mark.parametrize("n", [3, 4, 5])
@pytest.mark.parametrize("scatter,eps", [("atomic", 0.0), ("segmented", 0.0), ("atomic", 1.0),
                                         ("segmented", 1.0)])
def test_tiny_bodies_every_assembly_path(n, scatter, eps):
    """Lattices of 3^3, 4^3 and 5^3 nodes (48, 162 and 384 MPs): fewer MPs
    than the 512 workgroups of the fused shape-function kernel, so at most
    one MP per workgroup and most of them empty; with and without the
    stabilisation term (eps in units of mu h^2); 5 steps against the
    oracle."""
    w = W.elastic_cube(n=n, h=1.0, seed=0, steps=5)
    mu = w.material.E / (2 * (1 + w.material.nu))
    over = dict(eps_stab=eps * mu * w.h ** 2)
    st, p = _oracle_run(w, 5, **over)
    g, _ = _gpu_run(w, 5, scatter=scatter, **over)
    assert np.array_equal(g["offsets"], st.offsets) and np.array_equal(g["idx"], st.idx)
    errs = compare(gpu_fields(g, w.x_nodes, w.x_mp, p["T_r"]),
                   oracle_fields(st, w.x_nodes, w.x_mp, p["T_r"]))
    bad = {k: v for k, v in errs.items() if not v < FP64_TOL}
    assert not bad, bad
