"""HHO-hp: the HHO scheme with hybrid pressure (Section 2.3.2, Scheme 2) in matrix
form, its global system and its v&p-cond static condensation (test
infrastructure; see the package header).

Unknowns: cell velocities in P^{k+1}(T)^d and face velocities in P^k(F)^d (the
space V_h^{k+1,k}), cell pressures in P^k(T) and face pressures in P^k(F) (the
hybrid space V_h^{k,k}).  The viscous part is that of Scheme 1 with k' = k + 1:
potential reconstruction in P^{k+1}(T) (Section 2.2.1), face residual
r_TF v = pi_F^k(v_F - p v) - pi_T^{k+1}(v_T - p v) restricted to F (Section
2.2.3), which lives in P^{k+1}(F) and is integrated by quadrature, and the
symmetric Nitsche terms on Dirichlet faces.  The pressure-velocity coupling is
the hybrid one of the boxed terms.

Local scalar velocity unknowns are ordered cell first (dim P^{k+1}(T)
coefficients of the hierarchical orthonormal basis), then the faces of T in mesh
order (dim P^k(F) each); local pressure unknowns cell first (the first dim P^k(T)
modes of the same basis), then the faces.

Readings (the paper leaves them open or prints them ambiguously):
* the stabilisation term is read as R u . R v (the printed R v . R v is a typo);
* the printed mass residual carries no Dirichlet terms, while its momentum
  counterpart carries + sum_{F in F_T^D} (p_F, v_F . n_TF)_F; the mass residual
  is read as the transpose of the momentum coupling plus the datum, as in
  Scheme 1 with q_F in place of q_T:
  - (div u_T, q_T)_T + sum_F ((u_T - u_F) . n_TF, q_F)_F
  + sum_{F in F_T^D} ((u_F - g_D) . n_TF, q_F)_F,
  so the global matrix is symmetric and the face velocity of a Dirichlet face
  does not enter the mass balance (both readings reproduce polynomial solutions
  and give a pointwise divergence-free cell velocity);
* the Dirichlet datum in the Nitsche consistency term and the Neumann datum are
  read as in ``oracle.hho`` (same conventions);
* with a pure Dirichlet boundary the constant pressure (p_T = p_F = 1) spans the
  kernel; the solve borders the matrix with it, and the pressure is then
  shifted to zero mean over the cells.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .bases import CellBasis, dim_poly
from .geometry import cell_quadrature
from .hho import mesh_geometry


@dataclass
class LocalHP:
    d: int
    N1: int              # cell velocity modes per component (P^{k+1})
    nT: int              # cell pressure modes (P^k)
    nF: int              # face modes (P^k), velocity per component and pressure
    nfaces: int
    a: np.ndarray        # [nloc, nloc] scalar viscous matrix
    B: np.ndarray        # [d, npl, nloc] pressure-velocity coupling per velocity component
    rhs_u: np.ndarray    # [d, nloc]
    rhs_p: np.ndarray    # [npl]
    basis: CellBasis
    qpts: np.ndarray
    qw: np.ndarray

    @property
    def nloc(self):
        return self.N1 + self.nfaces * self.nF

    @property
    def npl(self):
        return self.nT + self.nfaces * self.nF


def local_hp(mesh, geo, c: int, eta: float, f_fn, gD_fn, gN_fn) -> LocalHP:
    """Local residuals of Scheme 2 on cell c as matrices: a (viscous, per
    component), B (coupling) and the data vectors."""
    d, k = mesh.dim, geo.k
    cg = geo.cells[c]
    xq, wq = cell_quadrature(mesh, cg, geo.faces, geo.qdeg)
    cb = CellBasis(cg.centroid, cg.diam, xq, wq, k + 1)
    N1, nT, nF = dim_poly(d, k + 1), dim_poly(d, k), dim_poly(d - 1, k)
    nfc = len(cg.faces)
    nloc, npl = N1 + nfc * nF, nT + nfc * nF
    phi, gphi = cb.values(xq), cb.grads(xq)

    # potential reconstruction p: (grad p v, grad w)_T = (grad v_T, grad w)_T
    # + sum_F (v_F - v_T, grad w . n_TF)_F for w in P^{k+1}(T), same mean as v_T
    K = np.einsum("q,qid,qjd->ij", wq, gphi, gphi)
    rhs = np.zeros((N1, nloc))
    rhs[:, :N1] = K
    faces = []
    for i, f in enumerate(cg.faces):
        n = cg.signs[i] * geo.faces[f].normal
        xf, wf = geo.face_q[f]
        psi = geo.face_basis[f].values(xf)                    # [qf, nF]
        phif = cb.values(xf)                                  # [qf, N1]
        gn = cb.grads(xf) @ n                                 # [qf, N1]
        cols = slice(N1 + i * nF, N1 + (i + 1) * nF)
        rhs[:, :N1] -= np.einsum("q,qi,qj->ij", wf, gn, phif)
        rhs[:, cols] += np.einsum("q,qi,qj->ij", wf, gn, psi)
        faces.append((i, f, n, cols, xf, wf, psi, phif, gn))
    R = np.zeros((N1, nloc))
    R[0, 0] = 1.0
    R[1:] = np.linalg.solve(K[1:, 1:], rhs[1:])

    a = R.T @ K @ R
    E_T = np.zeros((N1, nloc))
    E_T[:, :N1] = np.eye(N1)
    B = np.zeros((d, npl, nloc))
    rhs_u = np.zeros((d, nloc))
    rhs_p = np.zeros(npl)
    # -(q_T, div v_T)_T
    for cc in range(d):
        B[cc, :nT, :N1] -= np.einsum("q,qj,qi->ji", wq, phi[:, :nT], gphi[:, :, cc])
    for (i, f, n, cols, xf, wf, psi, phif, gn) in faces:
        hF = geo.faces[f].diam
        E_F = np.zeros((nF, nloc))
        E_F[:, cols] = np.eye(nF)
        Pi_F = np.einsum("q,qj,qi->ji", wf, psi, phif)        # [nF, N1] L2(F) projection of traces
        # face residual at the face's quadrature points: pi_F(v_F - p v) - (v_T - p v)|_F
        rq = psi @ (E_F - Pi_F @ R) - phif @ (E_T - R)        # [qf, nloc]
        a += np.einsum("q,qi,qj->ij", wf, rq, rq) / hF
        bc = mesh.face_bc[f]
        if bc == 1:
            Nn = np.einsum("q,qj,qi->ji", wf, psi, gn)        # [nF, N1] (psi_j, grad phi_i . n)_F
            a += -E_F.T @ Nn @ R - R.T @ Nn.T @ E_F + (eta / hF) * (E_F.T @ E_F)
        prow = slice(nT + i * nF, nT + (i + 1) * nF)
        for cc in range(d):
            # (q_F, v_T . n)_F - (q_F, v_F . n)_F, the second cancelled on Dirichlet faces
            B[cc, prow, :N1] += np.einsum("q,qj,qi->ji", wf, psi * n[cc], phif)
            if bc != 1:
                B[cc, prow, cols] -= np.einsum("q,qj,qi->ji", wf, psi * n[cc], psi)
        if bc == 1:
            g = gD_fn(xf)                                     # [qf, d]
            for cc in range(d):
                rhs_u[cc] -= R.T @ np.einsum("q,q,qi->i", wf, g[:, cc], gn)
                rhs_u[cc] += (eta / hF) * (E_F.T @ np.einsum("q,q,qj->j", wf, g[:, cc], psi))
            rhs_p[prow] += np.einsum("q,q,qj->j", wf, g @ n, psi)
        elif bc == 2:
            g = gN_fn(xf, np.repeat(n[None, :], len(xf), 0))
            for cc in range(d):
                rhs_u[cc] += E_F.T @ np.einsum("q,q,qj->j", wf, g[:, cc], psi)
    fq = f_fn(xq)
    for cc in range(d):
        rhs_u[cc, :N1] += np.einsum("q,q,qj->j", wq, fq[:, cc], phi)
    return LocalHP(d, N1, nT, nF, nfc, a, B, rhs_u, rhs_p, cb, xq, wq)


@dataclass
class HPProblem:
    mesh: object
    k: int
    eta: float
    geo: object
    locs: list
    NU: int      # face velocity unknowns: (face, component, mode)
    NP: int      # face pressure unknowns: (face, mode)
    NV: int      # cell velocity unknowns: (cell, component, mode)
    NQ: int      # cell pressure unknowns: (cell, mode)
    z: np.ndarray | None  # constant-pressure kernel vector (pure Dirichlet), full layout

    @property
    def nskel(self):
        return self.NU + self.NP

    @property
    def N(self):
        return self.NU + self.NP + self.NV + self.NQ


def default_eta_hp(mesh, k: int) -> float:
    """Penalty of the same form as Scheme 1's default with k' = k + 1."""
    mx = max(len(mesh.cell_faces(c)) for c in range(mesh.n_cells))
    return 4.0 * (k + 2) * (k + 1 + mesh.dim) / mesh.dim * mx


def build_hp(mesh, k: int, data, eta=None, qdeg=None) -> HPProblem:
    f_fn, gD_fn, gN_fn = data
    eta = default_eta_hp(mesh, k) if eta is None else eta
    geo = mesh_geometry(mesh, k, qdeg if qdeg is not None else 2 * k + 10)
    locs = [local_hp(mesh, geo, c, eta, f_fn, gD_fn, gN_fn) for c in range(mesh.n_cells)]
    d, nf, nc = mesh.dim, mesh.n_faces, mesh.n_cells
    N1, nT, nF = locs[0].N1, locs[0].nT, locs[0].nF
    P = HPProblem(mesh, k, eta, geo, locs, nf * d * nF, nf * nF, nc * d * N1, nc * nT, None)
    if not any(mesh.face_bc[f] == 2 for f in range(nf)):
        z = np.zeros(P.N)
        for f in range(nf):
            z[P.NU + f * nF] = np.sqrt(geo.faces[f].area)
        for c in range(nc):
            z[P.NU + P.NP + P.NV + c * nT] = np.sqrt(geo.cells[c].volume)
        P.z = z
    return P


def cell_system(P: HPProblem, c: int):
    """The cell's contribution to the global system: global indices (interior
    unknowns first: cell velocity, cell pressure; then the skeleton: face
    velocities, face pressures), the dense local matrix [[A, B^T], [B, 0]] and
    the right-hand side, in that order."""
    L, d = P.locs[c], P.mesh.dim
    N1, nT, nF = L.N1, L.nT, L.nF
    fs = list(P.geo.cells[c].faces)
    vel, pres = [], []      # (global index, component, local scalar index) / (global, local)
    for cc in range(d):
        for s in range(N1):
            vel.append((P.NU + P.NP + (c * d + cc) * N1 + s, cc, s))
    for j in range(nT):
        pres.append((P.NU + P.NP + P.NV + c * nT + j, j))
    nint = len(vel) + len(pres)
    for i, f in enumerate(fs):
        for cc in range(d):
            for j in range(nF):
                vel.append((f * d * nF + cc * nF + j, cc, N1 + i * nF + j))
    for i, f in enumerate(fs):
        for j in range(nF):
            pres.append((P.NU + f * nF + j, nT + i * nF + j))
    # order: interior velocity, interior pressure, face velocity, face pressure
    nvi = d * N1
    order = ([("v", e) for e in vel[:nvi]] + [("p", e) for e in pres[:nT]]
             + [("v", e) for e in vel[nvi:]] + [("p", e) for e in pres[nT:]])
    n = len(order)
    M = np.zeros((n, n))
    b = np.zeros(n)
    gidx = np.array([e[1][0] for e in order])
    for r, (kr, er) in enumerate(order):
        if kr == "v":
            _, ccr, sr = er
            b[r] = L.rhs_u[ccr, sr]
        else:
            b[r] = L.rhs_p[er[1]]
        for s, (ks, es) in enumerate(order):
            if kr == "v" and ks == "v":
                if er[1] == es[1]:
                    M[r, s] = L.a[er[2], es[2]]
            elif kr == "p" and ks == "v":
                M[r, s] = L.B[es[1], er[1], es[2]]
            elif kr == "v" and ks == "p":
                M[r, s] = L.B[er[1], es[1], er[2]]
    return gidx, nint, M, b


def assemble_full(P: HPProblem):
    rows, cols, vals = [], [], []
    b = np.zeros(P.N)
    for c in range(P.mesh.n_cells):
        g, _, M, bl = cell_system(P, c)
        r, s = np.nonzero(M)
        rows.append(g[r]); cols.append(g[s]); vals.append(M[r, s])
        np.add.at(b, g, bl)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(P.N, P.N))
    return A, b


def _bordered_solve(A, b, z):
    if z is None:
        return spla.splu(A.tocsc()).solve(b)
    n = A.shape[0]
    Ab = sp.bmat([[A, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]]).tocsc()
    return spla.splu(Ab).solve(np.append(b, 0.0))[:n]


def solve_uncondensed(P: HPProblem) -> np.ndarray:
    """All unknowns from the global system (sparse LU, bordered by the constant
    pressure when it spans the kernel)."""
    A, b = assemble_full(P)
    return _bordered_solve(A, b, P.z)


def condense_vp(P: HPProblem):
    """v&p-cond (Section 4.1.2 applied to Scheme 2): every cell's velocity and
    pressure unknowns are eliminated, leaving face velocities and face pressures.
    Returns the skeletal matrix, its right-hand side and the per-cell factors
    needed to recover the cell unknowns."""
    ns = P.nskel
    rows, cols, vals = [], [], []
    g = np.zeros(ns)
    keep = []
    for c in range(P.mesh.n_cells):
        gi, nint, M, bl = cell_system(P, c)
        MII, MIB, MBI, MBB = M[:nint, :nint], M[:nint, nint:], M[nint:, :nint], M[nint:, nint:]
        X = np.linalg.solve(MII, np.concatenate([MIB, bl[:nint, None]], axis=1))
        S = MBB - MBI @ X[:, :-1]
        gl = bl[nint:] - MBI @ X[:, -1]
        gb = gi[nint:]
        r, s = np.meshgrid(gb, gb, indexing="ij")
        rows.append(r.ravel()); cols.append(s.ravel()); vals.append(S.ravel())
        np.add.at(g, gb, gl)
        keep.append((gi, nint, X))
    Sg = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(ns, ns))
    return Sg, g, keep


def solve_condensed(P: HPProblem) -> np.ndarray:
    """Skeletal solve of the v&p-cond system, then recovery of the cell unknowns."""
    Sg, g, keep = condense_vp(P)
    zs = None if P.z is None else P.z[:P.nskel]
    xs = _bordered_solve(Sg, g, zs)
    x = np.zeros(P.N)
    x[:P.nskel] = xs
    for gi, nint, X in keep:
        x[gi[:nint]] = X[:, -1] - X[:, :-1] @ xs[gi[nint:]]
    return x


def normalise_pressure(P: HPProblem, x: np.ndarray) -> np.ndarray:
    """Shift cell and face pressures by one constant so that the cell pressures
    have zero mean over the domain."""
    if P.z is None:
        return x
    nT, nF = P.locs[0].nT, P.locs[0].nF
    tot = sum(x[P.NU + P.NP + P.NV + c * nT] * np.sqrt(P.geo.cells[c].volume) for c in range(P.mesh.n_cells))
    vol = sum(P.geo.cells[c].volume for c in range(P.mesh.n_cells))
    s = tot / vol
    y = x.copy()
    for c in range(P.mesh.n_cells):
        y[P.NU + P.NP + P.NV + c * nT] -= s * np.sqrt(P.geo.cells[c].volume)
    for f in range(P.mesh.n_faces):
        y[P.NU + f * nF] -= s * np.sqrt(P.geo.faces[f].area)
    return y


def cell_fields(P: HPProblem, x: np.ndarray, c: int):
    """Cell velocity [q, d], its gradient [q, d, d], its divergence [q] and the
    cell pressure [q] at the cell's quadrature points (with the weights)."""
    L, d = P.locs[c], P.mesh.dim
    N1, nT = L.N1, L.nT
    base = P.NU + P.NP + c * d * N1
    U = x[base:base + d * N1].reshape(d, N1)
    phi, gphi = L.basis.values(L.qpts), L.basis.grads(L.qpts)
    u = phi @ U.T
    gu = np.einsum("qid,ci->qcd", gphi, U)
    div = np.einsum("qcc->q", gu)
    pc = x[P.NU + P.NP + P.NV + c * nT:P.NU + P.NP + P.NV + (c + 1) * nT]
    p = phi[:, :nT] @ pc
    return u, gu, div, p, L.qw


def face_pressure(P: HPProblem, x: np.ndarray, f: int):
    """Face pressure at the face's quadrature points (with the weights)."""
    nF = P.locs[0].nF
    xf, wf = P.geo.face_q[f]
    psi = P.geo.face_basis[f].values(xf)
    return psi @ x[P.NU + f * nF:P.NU + (f + 1) * nF], xf, wf


def skeletal_order(P: HPProblem) -> np.ndarray:
    """perm[new] = old: the skeletal unknowns face by face, each face's d velocity
    components and then its pressure (P^k(F) modes each), the layout of a level
    with d + 1 components per face and no cell unknowns."""
    d, nF, nf = P.mesh.dim, P.locs[0].nF, P.mesh.n_faces
    perm = np.empty(P.nskel, dtype=np.int64)
    for f in range(nf):
        for cc in range(d + 1):
            for j in range(nF):
                old = f * d * nF + cc * nF + j if cc < d else P.NU + f * nF + j
                perm[(f * (d + 1) + cc) * nF + j] = old
    return perm


def multilevel_problem(P: HPProblem, degrees=None):
    """The v&p-cond skeletal system of Scheme 2 as a level hierarchy for the
    p-multilevel solver of Section 3: level l holds every face's d velocity
    components and its pressure in P^{k_l}(F); the prolongation injects the
    leading modes of the hierarchical face bases (Section 3.1) and the coarse
    operators are the Galerkin products, i.e. sub-blocks of the fine one.  The
    cell-patch Schwarz smoother then patches the faces of each cell.  Returns an
    ``oracle.solve.Problem`` (driven by ``oracle.solve.solve_fgmres`` and
    ``oracle.solve.solve_direct``) and the permutation of ``skeletal_order``."""
    from .solve import Problem
    from .system import LevelLayout, coarse_indices
    mesh, d, k = P.mesh, P.mesh.dim, P.k
    degrees = list(range(k, -1, -1)) if degrees is None else list(degrees)
    assert degrees[0] == k and all(a > b for a, b in zip(degrees, degrees[1:])) and degrees[-1] >= 0
    Sg, g, _ = condense_vp(P)
    perm = skeletal_order(P)
    S0 = Sg[perm][:, perm].tocsr()
    b = g[perm]
    lays = [LevelLayout(kl, d + 1, dim_poly(d - 1, kl), 0, mesh.n_faces, mesh.n_cells) for kl in degrees]
    S, idx = [S0], []
    for l in range(len(degrees) - 1):
        ii = coarse_indices(lays[l], lays[l + 1])
        idx.append(ii)
        S.append(S[-1][ii][:, ii].tocsr())
    zs = []
    for lay in lays:
        if P.z is None:
            zs.append(None)
            continue
        z = np.zeros(lay.N)
        for f in range(mesh.n_faces):
            z[(f * (d + 1) + d) * lay.nF] = np.sqrt(P.geo.faces[f].area)
        zs.append(z)
    return Problem(mesh, P.geo, k, "hp", degrees, P.eta, P.locs, None, lays, S, b, idx, zs), perm


def recover_from_skeleton(P: HPProblem, xs_ordered: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """All unknowns (layout of ``HPProblem``) from a skeletal solution in the
    order of ``skeletal_order``."""
    _, _, keep = condense_vp(P)
    x = np.zeros(P.N)
    x[perm] = xs_ordered
    for gi, nint, X in keep:
        x[gi[:nint]] = X[:, -1] - X[:, :-1] @ x[gi[nint:]]
    return x
