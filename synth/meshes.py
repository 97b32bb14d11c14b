"""Seeded mesh generators (topology + coordinates only).

A mesh is a pair (cells, faces) as in the paper's discrete setting (Section 2.1):
faces are line segments (d=2) or planar polygons (d=3); every cell lists the
faces on its boundary.  Storage is CSR:

* ``verts``      float64 [nv, d]
* ``face_ptr``   int64 [nf+1], ``face_vtx`` int64 -- vertices of each face.  In 2D a
  face is (a, b) with a < b; in 3D the polygon is listed cyclically starting at
  its lowest-index vertex.  This vertex order fixes each face's global
  orientation (tangent frame and reference normal).
* ``cell_ptr``   int64 [nc+1], ``cell_face`` int64 -- faces of each cell (2D:
  counter-clockwise).
* ``face_bc``    int8 [nf] -- 0 interior, 1 Dirichlet, 2 Neumann.

Generators:

* ``cartesian_quads`` -- uniform quadrilaterals on a box.
* ``voronoi_lloyd`` -- Lloyd-relaxed Voronoi polygons on the unit square, the
  cells clipped exactly to the square by mirroring the seeds across its sides.
* ``cartesian_hexes`` -- hexahedra on a (possibly graded) tensor grid.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


@dataclass
class Mesh:
    dim: int
    verts: np.ndarray
    face_ptr: np.ndarray
    face_vtx: np.ndarray
    cell_ptr: np.ndarray
    cell_face: np.ndarray
    face_bc: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return len(self.cell_ptr) - 1

    @property
    def n_faces(self) -> int:
        return len(self.face_ptr) - 1

    def cell_faces(self, c: int) -> np.ndarray:
        return self.cell_face[self.cell_ptr[c]:self.cell_ptr[c + 1]]

    def face_vertices(self, f: int) -> np.ndarray:
        return self.face_vtx[self.face_ptr[f]:self.face_ptr[f + 1]]

    def face_cells(self) -> np.ndarray:
        """[nf, 2] adjacent cells (second entry -1 on boundary faces)."""
        fc = -np.ones((self.n_faces, 2), dtype=np.int64)
        cnt = np.zeros(self.n_faces, dtype=np.int64)
        for c in range(self.n_cells):
            for f in self.cell_faces(c):
                if cnt[f] >= 2:
                    raise ValueError(f"face {f} has more than two cells")
                fc[f, cnt[f]] = c
                cnt[f] += 1
        return fc

    def with_bc(self, fn) -> "Mesh":
        """Return a copy whose boundary faces get ``fn(centroid) -> 1|2``."""
        bc = self.face_bc.copy()
        for f in range(self.n_faces):
            if bc[f] != 0:
                xv = self.verts[self.face_vertices(f)]
                bc[f] = fn(xv.mean(axis=0))
        return Mesh(self.dim, self.verts, self.face_ptr, self.face_vtx, self.cell_ptr,
                    self.cell_face, bc, self.name, dict(self.meta))


def _csr(lists):
    ptr = np.zeros(len(lists) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(x) for x in lists])
    idx = np.fromiter((v for x in lists for v in x), dtype=np.int64, count=int(ptr[-1]))
    return ptr, idx


def _boundary_flags(cell_face_lists, nf):
    cnt = np.zeros(nf, dtype=np.int64)
    for fl in cell_face_lists:
        for f in fl:
            cnt[f] += 1
    return np.where(cnt == 1, 1, 0).astype(np.int8)


def cartesian_quads(nx: int, ny: int | None = None, lo=(0.0, 0.0), hi=(1.0, 1.0)) -> Mesh:
    """Uniform nx-by-ny quadrilateral mesh of [lo, hi]; all boundary faces Dirichlet."""
    ny = nx if ny is None else ny
    xs = np.linspace(lo[0], hi[0], nx + 1)
    ys = np.linspace(lo[1], hi[1], ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    verts = np.stack([X.ravel(), Y.ravel()], axis=1)
    vid = lambda i, j: j * (nx + 1) + i  # noqa: E731
    faces = []
    hid = {}
    vid_e = {}
    for j in range(ny + 1):          # horizontal edges (i,j)-(i+1,j)
        for i in range(nx):
            hid[(i, j)] = len(faces)
            faces.append((vid(i, j), vid(i + 1, j)))
    for j in range(ny):              # vertical edges (i,j)-(i,j+1)
        for i in range(nx + 1):
            vid_e[(i, j)] = len(faces)
            faces.append((vid(i, j), vid(i, j + 1)))
    cells = []
    for j in range(ny):
        for i in range(nx):
            cells.append((hid[(i, j)], vid_e[(i + 1, j)], hid[(i, j + 1)], vid_e[(i, j)]))
    fptr, fvtx = _csr([sorted(f) for f in faces])
    cptr, cf = _csr(cells)
    return Mesh(2, verts, fptr, fvtx, cptr, cf, _boundary_flags(cells, len(faces)),
                name=f"quad{nx}x{ny}")


def _rings(vor, seeds, n):
    """Flattened vertex indices of the original cells, each cell's vertices sorted
    by angle around its seed (Voronoi cells are convex and contain their seed).
    Returns (ptr, idx)."""
    regs = [vor.regions[vor.point_region[i]] for i in range(n)]
    cnt = np.array([len(r) for r in regs])
    ptr = np.zeros(n + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(cnt)
    idx = np.fromiter((v for r in regs for v in r), dtype=np.int64, count=int(ptr[-1]))
    owner = np.repeat(np.arange(n), cnt)
    V = vor.vertices[idx]
    ang = np.arctan2(V[:, 1] - seeds[owner, 1], V[:, 0] - seeds[owner, 0])
    order = np.lexsort((ang, owner))
    return ptr, idx[order]


def _centroids(P, ptr):
    n = len(ptr) - 1
    owner = np.repeat(np.arange(n), np.diff(ptr))
    nxt = np.arange(len(P)) + 1
    nxt[ptr[1:] - 1] = ptr[:-1]
    x, y, xn, yn = P[:, 0], P[:, 1], P[nxt, 0], P[nxt, 1]
    cr = x * yn - xn * y
    a = np.bincount(owner, cr, n) / 2.0
    cx = np.bincount(owner, (x + xn) * cr, n) / (6 * a)
    cy = np.bincount(owner, (y + yn) * cr, n) / (6 * a)
    return np.stack([cx, cy], axis=1)


def _clipped_voronoi(seeds, band=None):
    """Voronoi diagram of the seeds plus their mirror images across the four sides
    of the unit square, so that the original cells tile the square exactly.  Only
    seeds within ``band`` of a side are mirrored (cells further inside cannot
    reach the boundary); the caller checks that every original cell stays inside."""
    from scipy.spatial import Voronoi
    parts = [seeds]
    for axis, val in ((0, 0.0), (0, 1.0), (1, 0.0), (1, 1.0)):
        m = np.ones(len(seeds), dtype=bool) if band is None else np.abs(seeds[:, axis] - val) < band
        q = seeds[m].copy()
        q[:, axis] = 2 * val - q[:, axis]
        parts.append(q)
    return Voronoi(np.concatenate(parts, 0))


def voronoi_lloyd(n_cells: int, seed: int, lloyd_iters: int = 20, merge_rel: float = 0.02) -> Mesh:
    """Lloyd-relaxed Voronoi mesh of the unit square with ``n_cells`` cells.

    Seeds: ``numpy.random.default_rng(seed).random((n_cells, 2))``.  Each Lloyd
    step moves every seed to the centroid of its (exactly clipped) cell.  Voronoi
    vertices closer than ``merge_rel / sqrt(n_cells)`` are merged (their mean
    position, boundary coordinates kept on the boundary), which removes the
    near-degenerate faces that nearly co-circular seeds create; every boundary
    face is Dirichlet.
    """
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    seeds = rng.random((n_cells, 2))
    n = n_cells
    for it in range(lloyd_iters + 1):
        vor = _clipped_voronoi(seeds, band=0.1)
        ptr, ring = _rings(vor, seeds, n)
        V = vor.vertices[ring]
        if ring.min() < 0 or V.min() < -1e-9 or V.max() > 1 + 1e-9:
            vor = _clipped_voronoi(seeds)
            ptr, ring = _rings(vor, seeds, n)
        if it == lloyd_iters:
            break
        seeds = np.clip(_centroids(vor.vertices[ring], ptr), 1e-12, 1 - 1e-12)
    used, ring_u = np.unique(ring, return_inverse=True)
    P = np.clip(vor.vertices[used], 0.0, 1.0)
    P[np.abs(P) < 1e-12] = 0.0
    P[np.abs(P - 1) < 1e-12] = 1.0
    tol = merge_rel / np.sqrt(n_cells)
    rep = np.arange(len(P))

    def root(a):
        while rep[a] != a:
            rep[a] = rep[rep[a]]
            a = rep[a]
        return a
    for a, b in sorted(cKDTree(P).query_pairs(tol)):
        ra, rb = root(a), root(b)
        if ra != rb:
            rep[max(ra, rb)] = min(ra, rb)
    rep = np.array([root(a) for a in range(len(P))])
    uniq, grp = np.unique(rep, return_inverse=True)
    cnt = np.bincount(grp)
    verts = np.stack([np.bincount(grp, P[:, j]) / cnt for j in range(2)], axis=1)
    for j in range(2):
        for val in (0.0, 1.0):
            on = np.zeros(len(uniq), dtype=bool)
            on[grp[P[:, j] == val]] = True
            verts[on, j] = val
    vid = grp[ring_u]
    edge_id = {}
    faces = []
    cells = []
    for i in range(n):
        ring_i = []
        for v in vid[ptr[i]:ptr[i + 1]]:
            if not ring_i or ring_i[-1] != v:
                ring_i.append(int(v))
        while len(ring_i) > 1 and ring_i[0] == ring_i[-1]:
            ring_i.pop()
        X = verts[ring_i]
        area2 = np.sum(X[:, 0] * np.roll(X[:, 1], -1) - np.roll(X[:, 0], -1) * X[:, 1])
        if area2 < 0:
            ring_i = ring_i[::-1]
        fl = []
        for a, b in zip(ring_i, ring_i[1:] + ring_i[:1]):
            e = (min(a, b), max(a, b))
            if e not in edge_id:
                edge_id[e] = len(faces)
                faces.append(e)
            fl.append(edge_id[e])
        cells.append(fl)
    fptr, fvtx = _csr(faces)
    cptr, cf = _csr(cells)
    m = Mesh(2, verts, fptr, fvtx, cptr, cf, _boundary_flags(cells, len(faces)),
             name=f"voronoi{n_cells}_s{seed}")
    flen = np.linalg.norm(verts[fvtx[1::2]] - verts[fvtx[0::2]], axis=1)
    m.meta.update(lloyd_iters=lloyd_iters, seed=seed, merge_tol=float(tol),
                  min_face_len=float(flen.min()), mean_face_len=float(flen.mean()))
    return m


def cartesian_hexes(n: int, coords=None) -> Mesh:
    """n^3 hexahedra on the unit cube (or on the tensor grid ``coords=(xs, ys, zs)``)."""
    if coords is None:
        xs = ys = zs = np.linspace(0.0, 1.0, n + 1)
    else:
        xs, ys, zs = (np.asarray(c, dtype=np.float64) for c in coords)
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    vid = lambda i, j, k: (k * (ny + 1) + j) * (nx + 1) + i  # noqa: E731
    faces = []
    fidx = {}

    def add(key, ring):
        r = list(ring)
        s = int(np.argmin(r))
        r = r[s:] + r[:s]
        fidx[key] = len(faces)
        faces.append(r)

    for k in range(nz):
        for j in range(ny):
            for i in range(nx + 1):   # x-normal faces
                add(("x", i, j, k), [vid(i, j, k), vid(i, j + 1, k), vid(i, j + 1, k + 1), vid(i, j, k + 1)])
    for k in range(nz):
        for j in range(ny + 1):
            for i in range(nx):       # y-normal faces
                add(("y", i, j, k), [vid(i, j, k), vid(i + 1, j, k), vid(i + 1, j, k + 1), vid(i, j, k + 1)])
    for k in range(nz + 1):
        for j in range(ny):
            for i in range(nx):       # z-normal faces
                add(("z", i, j, k), [vid(i, j, k), vid(i + 1, j, k), vid(i + 1, j + 1, k), vid(i, j + 1, k)])
    cells = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                cells.append([fidx[("x", i, j, k)], fidx[("x", i + 1, j, k)],
                              fidx[("y", i, j, k)], fidx[("y", i, j + 1, k)],
                              fidx[("z", i, j, k)], fidx[("z", i, j, k + 1)]])
    fptr, fvtx = _csr(faces)
    cptr, cf = _csr(cells)
    return Mesh(3, verts, fptr, fvtx, cptr, cf, _boundary_flags(cells, len(faces)),
                name=f"hex{nx}x{ny}x{nz}")


def graded_coords(n: int, seed: int, jitter: float = 0.05):
    """Grid planes at Gauss-Lobatto-like (Chebyshev-Lobatto) positions, randomly
    displaced by ``jitter`` times the local spacing (grading recipe of Section 5.1)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(3):
        t = 0.5 - 0.5 * np.cos(np.pi * np.arange(n + 1) / n)
        d = np.diff(t)
        t[1:-1] += jitter * rng.uniform(-1, 1, n - 1) * np.minimum(d[:-1], d[1:])
        out.append(t)
    return tuple(out)


def mesh_stats(m: Mesh) -> dict:
    nfc = np.diff(m.cell_ptr)
    return {"name": m.name, "dim": m.dim, "cells": m.n_cells, "faces": m.n_faces,
            "boundary_faces": int((m.face_bc != 0).sum()),
            "faces_per_cell_mean": float(nfc.mean()), "faces_per_cell_max": int(nfc.max()),
            **m.meta}
