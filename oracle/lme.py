"""Local max-ent (LME) shape functions (Sec. 2.3, LME equation).

For a material point x_p with support nodes x_I, d_I = x_p - x_I,

    Z_I = exp(-beta |d_I|^2 + lambda . d_I),  Z = sum_I Z_I,  N_I = Z_I / Z,

with the multiplier lambda fixed by first-order consistency
sum_I N_I d_I = 0, found by Newton-Raphson.  lambda minimises the convex
function log Z(lambda): its gradient is r = sum N_I d_I and its Hessian is
J = sum N_I d_I (x) d_I - r (x) r.  Readings adopted where the paper is silent:

* start from the previous multiplier (0 at t = 0); Newton step -J^{-1} r;
  Armijo backtracking on log Z (sufficient-decrease factor 1e-4 plus a
  round-off allowance of 1e-12 (1 + |log Z|), so that steps taken at the
  level of rounding are not rejected; up to 30 halvings); stop when
  |r|_2 <= tol; give up after ``max_iter`` iterations;
* exponentials are shifted by the largest exponent (same N, no overflow);
* the gradient is not printed in the paper.  Differentiating r(x, lambda(x))
  = 0 gives grad lambda = 2 beta 1 - J^{-1}, hence
  grad N_I = -N_I J^{-1} d_I.

Arrays are padded to the longest support (K_max) with a validity mask.
Works for float64 and, for complex-step derivatives, complex128 (decisions
are taken on real parts).
"""
from __future__ import annotations

import numpy as np


class LMENotConverged(RuntimeError):
    def __init__(self, mp_index):
        super().__init__(f"LME Newton did not converge at material point {mp_index}")
        self.mp_index = mp_index


def padded_pairs(offsets, idx):
    """(n_mp, K_max) pair ids and mask for CSR support lists."""
    offsets = np.asarray(offsets, np.int64)
    K = np.diff(offsets)
    kmax = int(K.max()) if K.size else 0
    col = np.arange(kmax)
    mask = col[None, :] < K[:, None]
    pair = offsets[:-1, None] + col[None, :]
    pair = np.where(mask, pair, 0)
    return pair, mask


def _evaluate(prior, d, mask, lam):
    """log Z, r, J and N at multiplier ``lam`` for a block of MPs."""
    f = prior + np.einsum("pki,pi->pk", d, lam)
    fmax = np.where(mask, f.real, -np.inf).max(axis=1)
    e = np.where(mask, np.exp(f - fmax[:, None]), 0.0)
    Z = e.sum(axis=1)
    N = e / Z[:, None]
    r = np.einsum("pk,pki->pi", N, d)
    S = np.einsum("pk,pki,pkj->pij", N, d, d)
    J = S - r[:, :, None] * r[:, None, :]
    logZ = np.log(Z) + fmax
    return logZ, r, J, N


def lme_solve(d, prior, mask, lam0, tol, max_iter=50, extra_iter=0):
    """Damped Newton for lambda on padded supports.

    d: (n, K, 3) offsets x_p - x_I, prior: (n, K) = -beta |d|^2.
    Returns lambda (n, 3), N (n, K), J (n, 3, 3) at the solution.
    ``extra_iter`` undamped Newton steps are taken after convergence (used by
    the complex-step variant so that the imaginary part converges as well).
    """
    n = d.shape[0]
    lam = np.array(lam0, dtype=np.result_type(d, lam0), copy=True)
    logZ, r, J, N = _evaluate(prior, d, mask, lam)
    extra_left = np.full(n, extra_iter)
    for _ in range(max_iter + extra_iter):
        conv = np.sqrt((r.real ** 2).sum(axis=1)) <= tol
        polish = conv & (extra_left > 0)
        step = ~conv | polish
        if not step.any():
            break
        extra_left[polish] -= 1
        a = np.nonzero(step)[0]
        # J is symmetric positive definite while x_p lies inside the hull of
        # its nodes; a degenerate J means the multiplier has run away
        detJ = np.linalg.det(J[a].real)
        scale = np.einsum("pii->p", J[a].real) ** 3
        bad = ~(detJ > 1e-30 * scale) | ~np.isfinite(detJ)
        if bad.any():
            raise LMENotConverged(int(a[np.nonzero(bad)[0][0]]))
        delta = -np.linalg.solve(J[a], r[a][:, :, None])[:, :, 0]
        slope = (r[a] * delta).sum(axis=1).real
        t = np.ones(a.size)
        pending = np.ones(a.size, dtype=bool)
        for halving in range(31):
            k = np.nonzero(pending)[0]
            if k.size == 0:
                break
            rows = a[k]
            trial = lam[rows] + t[k, None] * delta[k]
            lz, rr, JJ, NN = _evaluate(prior[rows], d[rows], mask[rows], trial)
            # Armijo test on log Z; polishing steps and the last halving are
            # taken as they are
            lz0 = logZ[rows].real
            ok = (lz.real <= lz0 + 1e-4 * t[k] * slope[k] + 1e-12 * (1.0 + np.abs(lz0))) \
                | polish[rows] | (halving == 30)
            acc = rows[ok]
            lam[acc] = trial[ok]
            logZ = logZ.astype(lz.dtype, copy=False)
            logZ[acc], r[acc], J[acc], N[acc] = lz[ok], rr[ok], JJ[ok], NN[ok]
            pending[k[ok]] = False
            t[k[~ok]] *= 0.5
    bad = np.nonzero(~(np.sqrt((r.real ** 2).sum(axis=1)) <= tol))[0]
    if bad.size:
        raise LMENotConverged(int(bad[0]))
    return lam, N, J


def lme_shape(x_nodes, x_mp, offsets, idx, beta, tol, max_iter=50, lam0=None,
              extra_iter=0):
    """Shape functions and gradients for every MP.

    Returns lam (n_mp, 3), N (P,), dN (P, 3) in CSR pair order.
    """
    x_nodes = np.asarray(x_nodes)
    x_mp = np.asarray(x_mp)
    n_mp = x_mp.shape[0]
    if n_mp == 0:                       # no material points: nothing to solve
        lam = np.zeros((0, 3)) if lam0 is None else np.asarray(lam0)
        return lam, np.zeros(0), np.zeros((0, 3))
    pair, mask = padded_pairs(offsets, idx)
    nodes = np.asarray(idx)[pair]
    d = x_mp[:, None, :] - x_nodes[nodes]
    d = np.where(mask[:, :, None], d, 0.0)
    prior = -beta * ((d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2])
    if lam0 is None:
        lam0 = np.zeros((n_mp, 3))
    lam, Npad, J = lme_solve(d, prior, mask, lam0, tol, max_iter, extra_iter)
    # grad N_I = -N_I J^{-1} d_I
    sol = np.linalg.solve(J, np.swapaxes(d, 1, 2))          # (n, 3, K)
    G = -Npad[:, :, None] * np.swapaxes(sol, 1, 2)          # (n, K, 3)
    P = int(offsets[-1])
    N = np.zeros(P, dtype=Npad.dtype)
    dN = np.zeros((P, 3), dtype=G.dtype)
    N[pair[mask]] = Npad[mask]
    dN[pair[mask]] = G[mask]
    return lam, N, dN


def lme_one(x_nodes_support, xp, beta, tol, max_iter=50, lam0=None):
    """Shape functions of a single MP with support node coordinates (K, 3)."""
    xs = np.asarray(x_nodes_support, np.float64)
    K = xs.shape[0]
    offsets = np.array([0, K], np.int64)
    idx = np.arange(K, dtype=np.int32)
    lam, N, dN = lme_shape(xs, np.asarray(xp, np.float64)[None, :], offsets, idx, beta, tol,
                           max_iter, None if lam0 is None else np.asarray(lam0)[None, :])
    return lam[0], N, dN
