"""Mesh geometry for the discrete setting of Section 2.1 (test infrastructure).

For every cell T: measure |T|, centroid x_T, diameter h_T, its faces F_T with
the outward unit normals n_TF.  For every face F: measure |F|, centroid x_F,
diameter h_F, a reference unit normal n_F and an orthonormal tangent frame fixed
by the face's stored vertex order (the global face orientation).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

from . import quadrature as Q


@dataclass
class FaceGeo:
    verts: np.ndarray      # [nv, d]
    area: float
    centroid: np.ndarray
    diam: float
    normal: np.ndarray     # reference unit normal
    tangents: np.ndarray   # [d-1, d]


@dataclass
class CellGeo:
    faces: np.ndarray      # global face ids, mesh order
    signs: np.ndarray      # +1 if n_F points out of T
    volume: float
    centroid: np.ndarray
    diam: float
    is_box: bool
    lo: np.ndarray
    hi: np.ndarray


def _diam(X):
    D = X[:, None, :] - X[None, :, :]
    return float(np.sqrt((D ** 2).sum(-1)).max())


def face_geometry(mesh, f: int) -> FaceGeo:
    X = mesh.verts[mesh.face_vertices(f)]
    if mesh.dim == 2:
        t = X[1] - X[0]
        L = float(np.linalg.norm(t))
        t = t / L
        n = np.array([t[1], -t[0]])
        return FaceGeo(X, L, 0.5 * (X[0] + X[1]), L, n, t[None, :])
    # planar polygon: Newell normal, area and centroid from a fan
    nrm = np.zeros(3)
    for i in range(len(X)):
        a, b = X[i], X[(i + 1) % len(X)]
        nrm += np.cross(a, b)
    area = 0.5 * np.linalg.norm(nrm)
    n = nrm / np.linalg.norm(nrm)
    c0 = X.mean(axis=0)
    cen = np.zeros(3)
    for i in range(len(X)):
        a, b = X[i], X[(i + 1) % len(X)]
        ar = 0.5 * np.linalg.norm(np.cross(a - c0, b - c0))
        cen += ar * (c0 + a + b) / 3.0
    cen /= area
    t1 = X[1] - X[0]
    t1 = t1 / np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    return FaceGeo(X, float(area), cen, _diam(X), n, np.stack([t1, t2]))


def cell_geometry(mesh, c: int, fgeo) -> CellGeo:
    faces = mesh.cell_faces(c)
    if mesh.dim == 2:
        X = np.concatenate([fgeo[f].verts for f in faces])
        ring = _ring2d(mesh, faces)
        x, y = ring[:, 0], ring[:, 1]
        xn, yn = np.roll(x, -1), np.roll(y, -1)
        cr = x * yn - xn * y
        vol = 0.5 * cr.sum()
        cen = np.array([((x + xn) * cr).sum(), ((y + yn) * cr).sum()]) / (6 * vol)
        vol = abs(vol)
    else:
        X = np.concatenate([fgeo[f].verts for f in faces])
        pts, w = Q.polyhedron([fgeo[f].verts for f in faces], 1)
        vol = float(w.sum())
        cen = (w[:, None] * pts).sum(0) / vol
    signs = np.array([1.0 if np.dot(fgeo[f].centroid - cen, fgeo[f].normal) > 0 else -1.0 for f in faces])
    lo, hi = X.min(axis=0), X.max(axis=0)
    is_box = False
    if mesh.dim == 3:
        is_box = bool(np.all(np.isclose(X, lo) | np.isclose(X, hi)) and
                      np.isclose(vol, np.prod(hi - lo)))
    return CellGeo(faces, signs, float(vol), cen, _diam(X), is_box, lo, hi)


def _ring2d(mesh, faces):
    """Counter-clockwise vertex ring of a 2D cell from its (ordered) faces."""
    segs = [tuple(mesh.face_vertices(f)) for f in faces]
    ring = []
    for i, (a, b) in enumerate(segs):
        na, nb = segs[(i + 1) % len(segs)]
        shared = a if a in (na, nb) else b
        ring.append(shared)
    # ring[i] is the vertex between face i and face i+1
    return mesh.verts[np.array(ring)]


def cell_quadrature(mesh, cg: CellGeo, fgeo, deg: int):
    if mesh.dim == 2:
        return Q.polygon(_ring2d(mesh, cg.faces), deg)
    if cg.is_box:
        return Q.box(cg.lo, cg.hi, deg)
    return Q.polyhedron([fgeo[f].verts for f in cg.faces], deg)


def face_quadrature(mesh, fg: FaceGeo, deg: int):
    if mesh.dim == 2:
        return Q.segment(fg.verts[0], fg.verts[1], deg)
    return Q.polygon(fg.verts, deg)
