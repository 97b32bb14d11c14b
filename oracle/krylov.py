"""Krylov solvers of Section 3.3 (test infrastructure; see package header).

* ``gmres_steps``: a fixed number m of right-preconditioned GMRES iterations from
  a given iterate (the smoother of the V-cycle; the paper uses "a few" such
  iterations, two in Section 5.2.2).  Arnoldi with classical Gram-Schmidt
  applied twice; the iterate update is the least-squares minimiser of the
  residual over the Krylov space, computed with ``numpy.linalg.lstsq``.
* ``gmres_solve``: the same iteration with restarts, run to a relative residual
  (used for the coarsest level in 3D, Section 5.2.2).
* ``fgmres``: flexible GMRES (the outer solver), a new preconditioner
  application per iteration, stopping on the explicitly recomputed true
  relative residual.

Readings: right preconditioning for the smoother, x0 = 0, restart 30 and
CGS2 for FGMRES (the paper states none of these).
"""
from __future__ import annotations

import numpy as np


def _cgs2(V, w):
    h = np.array([np.dot(v, w) for v in V])
    w = w - sum(hi * v for hi, v in zip(h, V))
    h2 = np.array([np.dot(v, w) for v in V])
    w = w - sum(hi * v for hi, v in zip(h2, V))
    return h + h2, w


def _lsq(H, beta):
    e1 = np.zeros(H.shape[0])
    e1[0] = beta
    y = np.linalg.lstsq(H, e1, rcond=None)[0]
    return y, float(np.linalg.norm(e1 - H @ y))


def gmres_steps(A, M, x, r0, m: int, project=None, tiny=1e-300):
    """x + Z y after m right-preconditioned GMRES iterations from residual r0.
    ``A``, ``M`` are callables; ``project`` (optional) is applied to M(v)."""
    beta = float(np.linalg.norm(r0))
    if beta <= tiny:
        return x.copy()
    V, Z = [r0 / beta], []
    H = np.zeros((m + 1, m))
    n = 0
    for j in range(m):
        z = M(V[j])
        if project is not None:
            z = project(z)
        Z.append(z)
        h, w = _cgs2(V, A(z))
        H[:j + 1, j] = h
        H[j + 1, j] = np.linalg.norm(w)
        n = j + 1
        if H[j + 1, j] <= 1e-14 * beta:
            break
        V.append(w / H[j + 1, j])
    y, _ = _lsq(H[:n + 1, :n], beta)
    return x + sum(yi * zi for yi, zi in zip(y, Z))


def gmres_solve(A, M, b, rtol: float, restart: int, maxit: int, project=None):
    """Restarted right-preconditioned GMRES from x = 0; stops when the
    least-squares residual estimate is <= rtol * |b| or after maxit iterations.
    Returns (x, iterations)."""
    x = np.zeros_like(b)
    nb = float(np.linalg.norm(b))
    if nb == 0.0:
        return x, 0
    its = 0
    r = b.copy()
    while its < maxit:
        beta = float(np.linalg.norm(r))
        V, Z = [r / beta], []
        H = np.zeros((restart + 1, restart))
        n, res = 0, beta
        for j in range(restart):
            z = M(V[j])
            if project is not None:
                z = project(z)
            Z.append(z)
            h, w = _cgs2(V, A(z))
            H[:j + 1, j] = h
            H[j + 1, j] = np.linalg.norm(w)
            n = j + 1
            its += 1
            _, res = _lsq(H[:n + 1, :n], beta)
            if res <= rtol * nb or its >= maxit or H[j + 1, j] <= 1e-14 * beta:
                break
            V.append(w / H[j + 1, j])
        y, _ = _lsq(H[:n + 1, :n], beta)
        x = x + sum(yi * zi for yi, zi in zip(y, Z))
        if res <= rtol * nb:
            break
        r = b - A(x)
    return x, its


def fgmres(A, M, b, rtol: float, restart: int = 30, maxit: int = 1000, project=None):
    """Flexible GMRES (Section 3.3) from x = 0.  Returns
    (x, iterations, history, converged) where history[i] is the least-squares
    relative residual estimate after i iterations (history[0] = 1)."""
    x = np.zeros_like(b)
    nb = float(np.linalg.norm(b))
    hist = [1.0]
    if nb == 0.0:
        return x, 0, hist, True
    its = 0
    r = b.copy()
    converged = False
    while its < maxit:
        beta = float(np.linalg.norm(r))
        V, Z = [r / beta], []
        H = np.zeros((restart + 1, restart))
        n = 0
        for j in range(restart):
            z = M(V[j])
            if project is not None:
                z = project(z)
            Z.append(z)
            h, w = _cgs2(V, A(z))
            H[:j + 1, j] = h
            H[j + 1, j] = np.linalg.norm(w)
            n = j + 1
            its += 1
            _, res = _lsq(H[:n + 1, :n], beta)
            hist.append(res / nb)
            if res <= rtol * nb or its >= maxit or H[j + 1, j] <= 1e-14 * beta:
                break
            V.append(w / H[j + 1, j])
        y, _ = _lsq(H[:n + 1, :n], beta)
        x = x + sum(yi * zi for yi, zi in zip(y, Z))
        r = b - A(x)
        if np.linalg.norm(r) <= rtol * nb:
            converged = True
            break
    return x, its, hist, converged
