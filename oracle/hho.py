"""HHO-dp local operators in matrix form (test infrastructure; see package header).

Follows Section 2.2 (scalar potential reconstruction, face residuals) and
Section 2.3.1 (local residuals of Scheme 1, equal order k' = k) and writes them
as the local algebraic system of eq. def:HHOAB.  Local scalar unknowns are
ordered cell first (dim P^k(T) coefficients), then the faces of T in mesh order
(dim P^k(F) coefficients each).  By the block-structure remark of Section 4.1.1
the velocity matrix is the scalar matrix ``a`` repeated on each component.

Conventions and readings (the paper leaves them open):
* penalty eta is a run parameter;
* the Neumann datum g_N is the traction (grad u - p I) n;
* Dirichlet data enter the rows of every unknown reached by the Nitsche
  consistency term, cell rows included (the residual of eq. HHOdiscrMNT is
  followed, not the block labels of eq. def:HHOAB);
* the datum term g_D . (n . grad P v) of the fourth line of eq. HHOdiscrMNT is
  taken with the sign that makes the symmetric Nitsche terms consistent, i.e.
  the residual holds -(u_F - g_D) . (n . grad P v); with the printed sign the
  scheme would not reproduce polynomial solutions;
* quadrature exact to total degree ``qdeg`` (default 2k+8).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

from .bases import CellBasis, FaceBasis, dim_poly
from .geometry import face_geometry, cell_geometry, cell_quadrature, face_quadrature


@dataclass
class Geometry:
    faces: list
    cells: list
    face_q: list      # (pts, w) per face
    face_basis: list  # FaceBasis(k) per face
    k: int
    qdeg: int


def mesh_geometry(mesh, k: int, qdeg: int | None = None) -> Geometry:
    qdeg = 2 * k + 8 if qdeg is None else qdeg
    fgeo = [face_geometry(mesh, f) for f in range(mesh.n_faces)]
    cgeo = [cell_geometry(mesh, c, fgeo) for c in range(mesh.n_cells)]
    fq = [face_quadrature(mesh, fg, qdeg) for fg in fgeo]
    fb = [FaceBasis(fg, q[0], q[1], k) for fg, q in zip(fgeo, fq)]
    return Geometry(fgeo, cgeo, fq, fb, k, qdeg)


@dataclass
class LocalHHO:
    d: int
    nT: int
    nF: int
    nfaces: int
    a: np.ndarray        # [nloc, nloc] scalar viscous matrix (lines 1-2 of eq. HHOdiscrMNT)
    B: np.ndarray        # [d, nT, nloc] pressure-velocity coupling per component
    rhs_u: np.ndarray    # [d, nloc] momentum data (f, g_D, g_N terms)
    rhs_p: np.ndarray    # [nT] mass data (g_D . n term)
    R: np.ndarray        # [dim P^{k+1}, nloc] potential reconstruction
    basis: CellBasis
    qpts: np.ndarray
    qw: np.ndarray

    @property
    def nloc(self):
        return self.nT + self.nfaces * self.nF


def local_hho(mesh, geo: Geometry, c: int, eta: float, f_fn, gD_fn, gN_fn) -> LocalHHO:
    d, k = mesh.dim, geo.k
    cg = geo.cells[c]
    xq, wq = cell_quadrature(mesh, cg, geo.faces, geo.qdeg)
    cb = CellBasis(cg.centroid, cg.diam, xq, wq, k + 1)
    N1, nT, nF = dim_poly(d, k + 1), dim_poly(d, k), dim_poly(d - 1, k)
    nfc = len(cg.faces)
    nloc = nT + nfc * nF
    phi, gphi = cb.values(xq), cb.grads(xq)

    # --- scalar potential reconstruction (Section 2.2.1)
    K = np.einsum("q,qid,qjd->ij", wq, gphi, gphi)
    rhs = np.zeros((N1, nloc))
    rhs[:, :nT] = K[:, :nT]                                   # (grad v_T, grad w)_T
    face_data = []
    for i, f in enumerate(cg.faces):
        n = cg.signs[i] * geo.faces[f].normal
        xf, wf = geo.face_q[f]
        psi = geo.face_basis[f].values(xf)                    # [qf, nF]
        phif = cb.values(xf)                                  # [qf, N1]
        gn = cb.grads(xf) @ n                                 # [qf, N1] grad w . n_TF
        cols = slice(nT + i * nF, nT + (i + 1) * nF)
        rhs[:, :nT] -= np.einsum("q,qi,qj->ij", wf, gn, phif[:, :nT])   # -(v_T, grad w.n)_F
        rhs[:, cols] += np.einsum("q,qi,qj->ij", wf, gn, psi)           # (v_F, grad w.n)_F
        face_data.append((f, n, cols, xf, wf, psi, phif, gn))
    R = np.zeros((N1, nloc))
    R[0, 0] = 1.0                           # mean of p_T v equals mean of v_T (phi_0 constant)
    R[1:] = np.linalg.solve(K[1:, 1:], rhs[1:])

    # --- consistency: (grad p u, grad p v)_T
    a = R.T @ K @ R
    E_T = np.zeros((nT, nloc))
    E_T[:, :nT] = np.eye(nT)
    B = np.zeros((d, nT, nloc))
    rhs_u = np.zeros((d, nloc))
    rhs_p = np.zeros(nT)
    for (f, n, cols, xf, wf, psi, phif, gn) in face_data:
        hF = geo.faces[f].diam
        E_F = np.zeros((nF, nloc))
        E_F[:, cols] = np.eye(nF)
        Pi_F = np.einsum("q,qj,qi->ji", wf, psi, phif)        # [nF, N1] L2(F) projection of traces
        # face residual r_TF (Section 2.2.3): pi_F(v_F - p v) - pi_T^k(v_T - p v)|_F
        D = E_F - Pi_F @ R - Pi_F[:, :nT] @ (E_T - R[:nT])
        a += D.T @ D / hF
        bc = mesh.face_bc[f]
        if bc == 1:                                           # Nitsche terms on Dirichlet faces
            Nn = np.einsum("q,qj,qi->ji", wf, psi, gn)        # [nF, N1] (psi_j, grad phi_i . n)_F
            a += -E_F.T @ Nn @ R - R.T @ Nn.T @ E_F + (eta / hF) * (E_F.T @ E_F)
        # pressure-velocity coupling, line 3 of eq. HHOdiscrMNT (= line 1 of HHOdiscrCNT)
        for cc in range(d):
            B[cc, :, :nT] += np.einsum("q,qj,qi->ij", wf, phif[:, :nT] * n[cc], phif[:, :nT])
            B[cc, :, cols] += -np.einsum("q,qj,qi->ij", wf, psi * n[cc], phif[:, :nT])
            if bc == 1:
                B[cc, :, cols] += np.einsum("q,qj,qi->ij", wf, psi * n[cc], phif[:, :nT])
        # boundary data (line 4 of HHOdiscrMNT, line 2 of HHOdiscrCNT)
        if bc == 1:
            g = gD_fn(xf)                                     # [qf, d]
            for cc in range(d):
                rhs_u[cc] -= R.T @ np.einsum("q,q,qi->i", wf, g[:, cc], gn)
                rhs_u[cc] += (eta / hF) * (E_F.T @ np.einsum("q,q,qj->j", wf, g[:, cc], psi))
            rhs_p += np.einsum("q,q,qi->i", wf, g @ n, phif[:, :nT])
        elif bc == 2:
            g = gN_fn(xf, np.repeat(n[None, :], len(xf), 0))
            for cc in range(d):
                rhs_u[cc] += E_F.T @ np.einsum("q,q,qj->j", wf, g[:, cc], psi)
    # -(div v_T, q)_T
    for cc in range(d):
        B[cc, :, :nT] -= np.einsum("q,qj,qi->ij", wq, gphi[:, :nT, cc], phi[:, :nT])
    fq = f_fn(xq)
    for cc in range(d):
        rhs_u[cc, :nT] += np.einsum("q,q,qj->j", wq, fq[:, cc], phi[:, :nT])
    return LocalHHO(d, nT, nF, nfc, a, B, rhs_u, rhs_p, R, cb, xq, wq)


def vector_system(L: LocalHHO):
    """Full local matrices of eq. def:HHOAB with velocity unknowns
    U_T = (component c, mode j) -> c*nT + j and
    U_dT = (face i, component c, mode j) -> (i*d + c)*nF + j.
    Returns (A_TT, A_Td, A_dd, B_T, B_d, F_T, G_d, Ghat)."""
    d, nT, nF, nf = L.d, L.nT, L.nF, L.nfaces
    comp_T = np.repeat(np.arange(d), nT)
    sidx_T = np.tile(np.arange(nT), d)
    comp_d = np.array([c for i in range(nf) for c in range(d) for _ in range(nF)])
    sidx_d = np.array([nT + i * nF + j for i in range(nf) for c in range(d) for j in range(nF)])
    comp = np.concatenate([comp_T, comp_d])
    sidx = np.concatenate([sidx_T, sidx_d])
    A = np.where(comp[:, None] == comp[None, :], L.a[sidx[:, None], sidx[None, :]], 0.0)
    Bf = L.B[comp, :, sidx].T                    # [nT, nvel]
    rhs = L.rhs_u[comp, sidx]
    nU = d * nT
    return (A[:nU, :nU], A[:nU, nU:], A[nU:, nU:], Bf[:, :nU], Bf[:, nU:],
            rhs[:nU], rhs[nU:], L.rhs_p.copy())
