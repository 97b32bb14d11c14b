"""Global systems and the level hierarchy (test infrastructure; see package header).

Global unknown numbering (also the library's output layout):
* face velocity:   (face f, component c, mode j) -> (f*d + c)*nF + j
* v-cond pressure: (cell T, mode q)              -> nfaces*d*nF + T*nT + q
* v&p-cond:        (cell T, mean)                -> nfaces*d*nF + T
* uncond adds cell velocities after the faces:   (T, c, j) -> nfaces*d*nF + (T*d + c)*nT + j,
  then the pressures.

Assembly is the element-by-element sum of Section 2.3.1 (eq. HHOdisrcGlobalRes).
Coarse operators are the Galerkin projections of Section 3.2 / 4.2 computed
explicitly as P^T S P with the prolongation matrices P built from their
definition, and separately by sub-block extraction (Section 4.2).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np
import scipy.sparse as sp

from .bases import dim_poly
from .hho import LocalHHO, vector_system


def face_dofs(mesh, c, d, nF):
    fl = mesh.cell_faces(c)
    return np.array([(f * d + cc) * nF + j for f in fl for cc in range(d) for j in range(nF)])


def assemble_condensed(mesh, blocks, d, nF, nP):
    """Sum per-cell condensed (S, rhs) into the global sparse matrix."""
    nf = mesh.n_faces
    off = nf * d * nF
    N = off + mesh.n_cells * nP
    rows, cols, vals = [], [], []
    b = np.zeros(N)
    for c, (S, r) in enumerate(blocks):
        g = np.concatenate([face_dofs(mesh, c, d, nF), off + c * nP + np.arange(nP)])
        rows.append(np.repeat(g, len(g)))
        cols.append(np.tile(g, len(g)))
        vals.append(S.ravel())
        np.add.at(b, g, r)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    return A, b


def assemble_uncondensed(mesh, locs: list[LocalHHO]):
    d, nT, nF = locs[0].d, locs[0].nT, locs[0].nF
    nf, nc = mesh.n_faces, mesh.n_cells
    offU = nf * d * nF
    offP = offU + nc * d * nT
    N = offP + nc * nT
    rows, cols, vals = [], [], []
    b = np.zeros(N)
    for c, L in enumerate(locs):
        A_TT, A_Td, A_dd, B_T, B_d, F_T, G_d, Gh = vector_system(L)
        gT = offU + c * d * nT + np.arange(d * nT)
        gd = face_dofs(mesh, c, d, nF)
        gP = offP + c * nT + np.arange(nT)
        g = np.concatenate([gT, gd, gP])
        nU = d * nT
        M = np.block([[A_TT, A_Td, B_T.T], [A_Td.T, A_dd, B_d.T],
                      [B_T, B_d, np.zeros((nT, nT))]])
        rows.append(np.repeat(g, len(g)))
        cols.append(np.tile(g, len(g)))
        vals.append(M.ravel())
        np.add.at(b, g, np.concatenate([F_T, G_d, Gh]))
        del nU
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    return A, b


@dataclass
class LevelLayout:
    k: int
    d: int
    nF: int
    nP: int
    nfaces: int
    ncells: int

    @property
    def off(self):
        return self.nfaces * self.d * self.nF

    @property
    def N(self):
        return self.off + self.ncells * self.nP


def layout(mesh, k, cond):
    d = mesh.dim
    nP = dim_poly(d, k) if cond == "v" else 1
    return LevelLayout(k, d, dim_poly(d - 1, k), nP, mesh.n_faces, mesh.n_cells)


def prolongation(fine: LevelLayout, coarse: LevelLayout) -> sp.csr_matrix:
    """Algebraic prolongation I_{l+1}^{l} (Section 4.2): the transpose of the
    restriction matrix (int_X psi_i^{l+1} psi_j^{l}), which for hierarchical
    orthonormal bases is the unit-diagonal injection of the leading modes."""
    r, c = [], []
    for f in range(fine.nfaces):
        for cc in range(fine.d):
            for j in range(coarse.nF):
                r.append((f * fine.d + cc) * fine.nF + j)
                c.append((f * coarse.d + cc) * coarse.nF + j)
    for T in range(fine.ncells):
        for q in range(coarse.nP):
            r.append(fine.off + T * fine.nP + q)
            c.append(coarse.off + T * coarse.nP + q)
    return sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(fine.N, coarse.N))


def coarse_indices(fine: LevelLayout, coarse: LevelLayout) -> np.ndarray:
    """Fine-level index of every coarse unknown (sub-block extraction)."""
    P = prolongation(fine, coarse).tocsc()
    return P.indices[np.argsort(np.repeat(np.arange(coarse.N), np.diff(P.indptr)), kind="stable")]


def nullspace(mesh, geo, lay: LevelLayout):
    """Constant-pressure vector z (z_T = |T|^{1/2} on the mean mode) when there is
    no Neumann face, else None."""
    if np.any(mesh.face_bc == 2):
        return None
    z = np.zeros(lay.N)
    for T in range(lay.ncells):
        z[lay.off + T * lay.nP] = np.sqrt(geo.cells[T].volume)
    return z


def counts(mesh, k: int):
    """DOF and MNZ counts of Table tab:DOFsMNZsFormula, with the readings: v-cond
    face DOFs use d (not d+1), the v&p face/cell coupling uses dim P^{d-1}_k, and
    the face stencil factor (2 card - 1) is the exact number of faces of the
    cells sharing F (boundary faces included)."""
    d = mesh.dim
    nc, nf = mesh.n_cells, mesh.n_faces
    PT, PF = dim_poly(d, k), dim_poly(d - 1, k)
    fc = mesh.face_cells()
    card_TF = (fc >= 0).sum(axis=1)
    card_FT = np.diff(mesh.cell_ptr)
    sum_card_FT = card_FT.sum()
    # face stencil of F: distinct faces of the cells sharing F
    stencil = np.zeros(nf, dtype=np.int64)
    for f in range(nf):
        cells = fc[f][fc[f] >= 0]
        stencil[f] = sum(card_FT[c] for c in cells) - (len(cells) - 1)
    out = {
        "dof_uncond": nc * (d + 1) * PT + nf * d * PF,
        "dof_vp": nc + nf * d * PF,
        "dof_v": nc * PT + nf * d * PF,
        "dof_hp": nf * (d + 1) * PF,
        "dof_dg": nc * (d + 1) * PT,
        "mnz_vp": nc + sum_card_FT * d * PF + (stencil * d * d * PF * PF).sum()
        + (card_TF * d * PF).sum(),
        "mnz_hp": (stencil * (d + 1) ** 2 * PF * PF).sum(),
    }
    return {k_: int(v) for k_, v in out.items()}
