"""Pins of the oracle's LME shape functions (Sec. 2.3)."""
import numpy as np
import pytest

from oracle import lme, search
import otm_workloads as inputs


@pytest.fixture(scope="module")
def cube_shape(cube):
    off, idx = search.neighbors_bruteforce(cube.x_nodes, cube.x_mp, cube.r_list)
    lam, N, dN = lme.lme_shape(cube.x_nodes, cube.x_mp, off, idx, cube.beta, 1e-13 * cube.h)
    return off, idx, lam, N, dN


def _segsum(v, off):
    return np.add.reduceat(v, off[:-1], axis=0)


def test_partition_of_unity_and_linear_reproduction(cube, cube_shape):
    off, idx, lam, N, dN = cube_shape
    assert np.all(N > 0)
    assert np.abs(_segsum(N, off) - 1).max() < 1e-15 * 8
    xr = _segsum(N[:, None] * cube.x_nodes[idx], off)
    assert np.abs(xr - cube.x_mp).max() < 1e-13 * cube.h * 10


def test_gradient_identities(cube, cube_shape):
    # both identities hold up to J^{-1} r, r being the Newton residual
    # (|r| <= 1e-13 h) and |J^{-1}| <= ~10 / h^2 at corner material points
    off, idx, lam, N, dN = cube_shape
    assert np.abs(_segsum(dN, off)).max() < 1e-11 / cube.h
    outer = _segsum(cube.x_nodes[idx][:, :, None] * dN[:, None, :], off)
    assert np.abs(outer - np.eye(3)).max() < 1e-10


def test_gradient_matches_central_differences(cube, cube_shape):
    off, idx, lam, N, dN = cube_shape
    rng = np.random.default_rng(7)
    h = 1e-6 * cube.h
    worst = 0.0
    for p in rng.choice(cube.n_mp, 25, replace=False):
        nodes = cube.x_nodes[idx[off[p]:off[p + 1]]]
        g = dN[off[p]:off[p + 1]]
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            _, Np, _ = lme.lme_one(nodes, cube.x_mp[p] + e, cube.beta, 1e-14 * cube.h)
            _, Nm, _ = lme.lme_one(nodes, cube.x_mp[p] - e, cube.beta, 1e-14 * cube.h)
            fd = (Np - Nm) / (2 * h)
            worst = max(worst, np.abs(fd - g[:, a]).max() / np.abs(g).max())
    assert worst < 1e-7


def test_symmetric_lattice_closed_form():
    """MP at the centre of a perfect cubic node arrangement: lambda = 0 by
    symmetry and N_I = exp(-beta |d_I|^2) / sum."""
    h = 0.5
    g = np.arange(-3, 4) * h
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    beta = 4.0 / h ** 2
    r = h * np.sqrt(-np.log(1e-6) / 4.0)
    xp = np.zeros(3)
    nbr = search.neighbors_one(X, xp, r)
    lam, N, dN = lme.lme_one(X[nbr], xp, beta, 1e-13 * h, lam0=np.array([0.3, -0.2, 0.1]) / h)
    w = np.exp(-beta * (X[nbr] ** 2).sum(1))
    assert np.abs(lam).max() < 1e-10 / h
    assert np.abs(N - w / w.sum()).max() < 1e-14
    # and the gradient of a symmetric arrangement at its centre is
    # -N_I S^{-1} d_I with S = sum N d d^T = s 1 (cubic symmetry)
    s = (N * X[nbr][:, 0] ** 2).sum()
    assert np.abs(dN - (N[:, None] * X[nbr] / s)).max() < 1e-12 / h


def test_two_node_limit_is_linear_interpolation():
    """Along a line with two nodes the constrained max-ent functions reduce
    to the linear hat functions N = (x1 - x)/(x1 - x0), (x - x0)/(x1 - x0),
    whatever beta (first-order consistency fixes them).  Lifted to 3D with
    nodes off the line symmetric so the transverse multipliers vanish."""
    x0, x1 = 0.0, 1.0
    for xq in (0.1, 0.37, 0.5, 0.93):
        # 4 copies of each end node placed symmetrically around the axis
        eps = 1e-1
        ring = np.array([[0, eps, 0], [0, -eps, 0], [0, 0, eps], [0, 0, -eps]])
        X = np.concatenate([ring + [x0, 0, 0], ring + [x1, 0, 0]])
        lam, N, dN = lme.lme_one(X, np.array([xq, 0, 0]), 3.0, 1e-15)
        n1 = N[4:].sum()
        assert abs(n1 - (xq - x0) / (x1 - x0)) < 1e-13


def test_warm_start_reaches_same_solution(cube, cube_shape):
    off, idx, lam, N, dN = cube_shape
    lam2, N2, dN2 = lme.lme_shape(cube.x_nodes, cube.x_mp, off, idx, cube.beta,
                                  1e-13 * cube.h, lam0=lam * 0.9 + 0.01)
    assert np.abs(N2 - N).max() < 1e-13
    assert np.abs(dN2 - dN).max() < 1e-12


def test_nonconvergence_raises():
    """An MP outside the convex hull of its nodes has no consistent LME
    functions: the Newton iteration must report failure."""
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    with pytest.raises(lme.LMENotConverged):
        lme.lme_one(X, np.array([2.0, 2.0, 2.0]), 4.0, 1e-13, max_iter=50)
