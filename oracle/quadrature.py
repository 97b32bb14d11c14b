"""Quadrature rules (test infrastructure; see the package header).

The paper fixes no rule.  Rules used here are Gauss-Legendre on segments, the
collapsed (Duffy) product Gauss rule on triangles and tetrahedra, fan
sub-division of polygons / polyhedra from the vertex average, and tensor
Gauss-Legendre on axis-aligned boxes.  ``deg`` is the total polynomial degree
integrated exactly.
"""
from __future__ import annotations

import numpy as np


def gauss01(n: int):
    """n-point Gauss-Legendre rule on [0, 1] (exact to degree 2n-1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def segment(a: np.ndarray, b: np.ndarray, deg: int):
    t, w = gauss01(max(1, (deg + 2) // 2))
    pts = a[None, :] + t[:, None] * (b - a)[None, :]
    return pts, w * np.linalg.norm(b - a)


def triangle(v0, v1, v2, deg: int):
    """Collapsed rule x(s,t) = v0 + s[(v1-v0) + t(v2-v1)], Jacobian s*|J|."""
    n = max(1, (deg + 3) // 2)
    s, ws = gauss01(n)
    t, wt = gauss01(n)
    S, T = np.meshgrid(s, t, indexing="ij")
    W = np.outer(ws, wt) * S
    e1, e2 = v1 - v0, v2 - v1
    pts = v0[None, :] + S.ravel()[:, None] * (e1[None, :] + T.ravel()[:, None] * e2[None, :])
    if len(v0) == 2:
        jac = abs(e1[0] * e2[1] - e1[1] * e2[0])
    else:
        jac = np.linalg.norm(np.cross(e1, e2))
    return pts, W.ravel() * jac


def tetra(v0, v1, v2, v3, deg: int):
    n = max(1, (deg + 4) // 2)
    s, ws = gauss01(n)
    S, T, U = np.meshgrid(s, s, s, indexing="ij")
    W = (ws[:, None, None] * ws[None, :, None] * ws[None, None, :]) * S ** 2 * T
    e1, e2, e3 = v1 - v0, v2 - v1, v3 - v2
    S, T, U = S.ravel(), T.ravel(), U.ravel()
    pts = v0[None, :] + S[:, None] * (e1[None, :] + T[:, None] * (e2[None, :] + U[:, None] * e3[None, :]))
    return pts, W.ravel() * abs(np.linalg.det(np.stack([e1, e2, e3])))


def polygon(ring: np.ndarray, deg: int):
    """Fan from the vertex average; ``ring`` [nv, dim] is a convex polygon."""
    c = ring.mean(axis=0)
    P, W = [], []
    for i in range(len(ring)):
        p, w = triangle(c, ring[i], ring[(i + 1) % len(ring)], deg)
        P.append(p)
        W.append(w)
    return np.concatenate(P), np.concatenate(W)


def box(lo: np.ndarray, hi: np.ndarray, deg: int):
    n = max(1, (deg + 2) // 2)
    t, w = gauss01(n)
    grids = np.meshgrid(*[lo[j] + t * (hi[j] - lo[j]) for j in range(len(lo))], indexing="ij")
    wg = np.ones(1)
    for j in range(len(lo)):
        wg = np.multiply.outer(wg, w * (hi[j] - lo[j]))
    return np.stack([g.ravel() for g in grids], axis=1), wg.ravel()


def polyhedron(face_rings, deg: int):
    """Pyramids from the vertex average over fan triangles of every face."""
    allv = np.concatenate(face_rings)
    c = allv.mean(axis=0)
    P, W = [], []
    for ring in face_rings:
        fc = ring.mean(axis=0)
        for i in range(len(ring)):
            p, w = tetra(c, fc, ring[i], ring[(i + 1) % len(ring)], deg)
            P.append(p)
            W.append(w)
    return np.concatenate(P), np.concatenate(W)
