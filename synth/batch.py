"""Seeded batches of independent problems (inputs only, no method arithmetic).

A batch member is a Cartesian mesh of the unit square with a random side and
HHO degree; members are placed side by side (member i shifted by ``width * i``
along x) so that one data callback on their disjoint union can tell them apart.
"""
from __future__ import annotations

import copy
import numpy as np


def batch_spec(n: int = 256, seed: int = 4, side=(16, 96), degree=(1, 4)):
    """[(side, k, forcing seed)] with side ~ U{side}, k ~ U{degree}, forcing seed 4000 + i."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(side[0], side[1] + 1, size=n)
    ks = rng.integers(degree[0], degree[1] + 1, size=n)
    return [(int(s), int(k), 4000 + i) for i, (s, k) in enumerate(zip(sides, ks))]


def shifted(mesh, dx: float):
    """The mesh moved by dx along x."""
    m = copy.copy(mesh)
    m.verts = mesh.verts.copy()
    m.verts[:, 0] += dx
    return m


def region_fields(fields, dim: int, width: float):
    """(f, g_D, g_N) callbacks of a union whose member i occupies x in
    [width*i, width*i + 1]: each point is handed, shifted back, to the data of its member."""
    nmem = len(fields)

    def make(kind):
        if all(fl[kind] is None for fl in fields):
            return None

        def cb(x, *rest):
            out = np.zeros((x.shape[0], dim))
            idx = np.clip(np.floor(x[:, 0] / width + 1e-9).astype(int), 0, nmem - 1)
            order = np.argsort(idx, kind="stable")        # the points of each member, contiguous
            bounds = np.searchsorted(idx[order], np.arange(nmem + 1))
            for i in range(nmem):
                fn = fields[i][kind]
                sel = order[bounds[i]:bounds[i + 1]]
                if fn is None or sel.size == 0:
                    continue
                y = x[sel]
                y[:, 0] -= width * i
                out[sel] = fn(y, *[r[sel] for r in rest])
            return out
        return cb
    return make(0), make(1), make(2)


def disjoint_union(meshes):
    """One mesh holding the given meshes side by side, unconnected (member i's
    vertices, faces and cells follow those of members 0..i-1, in their order)."""
    from .meshes import Mesh
    dim = meshes[0].dim
    verts, fptr, fvtx, cptr, cface, bc = [], [0], [], [0], [], []
    nv = nf = 0
    for m in meshes:
        assert m.dim == dim
        verts.append(m.verts)
        fvtx.append(m.face_vtx + nv)
        fptr.extend((m.face_ptr[1:] + fptr[-1]).tolist())
        cface.append(m.cell_face + nf)
        cptr.extend((m.cell_ptr[1:] + cptr[-1]).tolist())
        bc.append(m.face_bc)
        nv += len(m.verts)
        nf += m.n_faces
    return Mesh(dim, np.concatenate(verts), np.array(fptr, dtype=np.int64), np.concatenate(fvtx),
                np.array(cptr, dtype=np.int64), np.concatenate(cface), np.concatenate(bc).astype(np.int8),
                "union")
