"""End-to-end oracle driver (test infrastructure; see package header).

``build`` forms the local HHO-dp operators of every cell, condenses them
(v-cond, eq. ST.1, or v&p-cond, eq. ST.2), assembles the global system and the
level hierarchy k_0 > k_1 > ... > k_L (Section 3, with coarse operators inherited
by Galerkin projection of the condensed operator, Section 4.2).  ``solve_direct``
gives the exact discrete solution; ``solve_fgmres`` runs FGMRES preconditioned
by one V-cycle per iteration (Section 3.3).  ``errors`` evaluates the error
measures of Section 5.2.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .bases import dim_poly
from .condense import condense_v, condense_vp, recover_v, recover_vp
from .hho import mesh_geometry, local_hho
from .ilu import ILU0
from .krylov import fgmres
from .multilevel import Hierarchy, Schwarz
from .system import (assemble_condensed, coarse_indices, face_dofs, layout, nullspace)


def default_eta(mesh, k: int) -> float:
    """Penalty reading: eta = 4 (k+1)(k+d)/d * max_T card(F_T)."""
    d = mesh.dim
    return 4.0 * (k + 1) * (k + d) / d * int(np.diff(mesh.cell_ptr).max())


@dataclass
class Problem:
    mesh: object
    geo: object
    k: int
    cond: str
    degrees: list
    eta: float
    locs: list
    blocks: list
    lays: list
    S: list
    b: np.ndarray
    idx: list
    z: list


def build(mesh, k: int, cond: str, data, degrees=None, eta=None, qdeg=None) -> Problem:
    f_fn, gD_fn, gN_fn = data
    degrees = list(range(k, -1, -1)) if degrees is None else list(degrees)
    assert degrees[0] == k and all(a > b for a, b in zip(degrees, degrees[1:])) and degrees[-1] >= 0
    eta = default_eta(mesh, k) if eta is None else eta
    geo = mesh_geometry(mesh, k, qdeg)
    locs = [local_hho(mesh, geo, c, eta, f_fn, gD_fn, gN_fn) for c in range(mesh.n_cells)]
    cfun = condense_v if cond == "v" else condense_vp
    blocks = [cfun(L) for L in locs]
    lays = [layout(mesh, kl, cond) for kl in degrees]
    S0, b = assemble_condensed(mesh, blocks, mesh.dim, lays[0].nF, lays[0].nP)
    S, idx = [S0], []
    for l in range(len(degrees) - 1):
        ii = coarse_indices(lays[l], lays[l + 1])
        idx.append(ii)
        S.append(S[-1][ii][:, ii].tocsr())
    z = [nullspace(mesh, geo, lay) for lay in lays]
    return Problem(mesh, geo, k, cond, degrees, eta, locs, blocks, lays, S, b, idx, z)


def project_out(z):
    if z is None:
        return lambda v: v
    zz = float(z @ z)
    return lambda v: v - (z @ v) / zz * z


def solve_direct(P: Problem) -> np.ndarray:
    """Exact discrete solution of the condensed system; with a pure Dirichlet
    boundary the constant-pressure mode is removed by bordering with z."""
    S, b, z = P.S[0], P.b, P.z[0]
    if z is None:
        return spla.spsolve(S.tocsc(), b)
    Sb = sp.bmat([[S, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]]).tocsc()
    return spla.spsolve(Sb, np.concatenate([b, [0.0]]))[:S.shape[0]]


def hierarchy(P: Problem, smooth_its=2, coarse="direct", coarse_rtol=1e-3,
              coarse_restart=30, coarse_maxit=500, smoother="schwarz") -> Hierarchy:
    """smoother: "schwarz" (the cell-patch preconditioner the GPU library uses)
    or "ilu" (zero-fill ILU in the natural ordering, the paper's, Section 3.3)."""
    if smoother == "schwarz":
        precs = [Schwarz(S, P.mesh, lay) for S, lay in zip(P.S, P.lays)]
    elif smoother == "ilu":
        precs = [ILU0(S) for S in P.S]
    else:
        raise ValueError(f"unknown smoother {smoother!r}")
    H = Hierarchy(P.S, P.idx, precs, P.z, smooth_its, coarse, coarse_rtol, coarse_restart, coarse_maxit)
    H.nface_dofs = [lay.off for lay in P.lays]
    H.dim = P.mesh.dim
    return H


def solve_fgmres(P: Problem, rtol=1e-8, restart=30, maxit=1000, H: Hierarchy | None = None, **hk):
    H = hierarchy(P, **hk) if H is None else H
    proj = project_out(P.z[0])
    b = proj(P.b)
    S0 = P.S[0]
    x, its, hist, conv = fgmres(lambda v: S0 @ v, lambda v: H.vcycle(0, v), b, rtol,
                                restart, maxit, project=proj)
    return proj(x), its, hist, conv


def normalise_pressure(P: Problem, x: np.ndarray) -> np.ndarray:
    """Shift the pressure to zero mean when it is defined up to a constant."""
    z = P.z[0]
    return x if z is None else x - (z @ x) / (z @ z) * z


def recover(P: Problem, x: np.ndarray):
    """Cell velocities U_T [nc, d*nT] and full cell pressures [nc, nT]."""
    lay = P.lays[0]
    d, nF, nP = lay.d, lay.nF, lay.nP
    UT, PT = [], []
    for c, L in enumerate(P.locs):
        Ud = x[face_dofs(P.mesh, c, d, nF)]
        p = x[lay.off + c * nP: lay.off + (c + 1) * nP]
        if P.cond == "v":
            UT.append(recover_v(L, Ud, p))
            PT.append(p)
        else:
            u, pf = recover_vp(L, Ud, p[0])
            UT.append(u)
            PT.append(pf)
    return np.array(UT), np.array(PT)


def errors(P: Problem, x: np.ndarray, man) -> dict:
    """Errors of Section 5.2: velocity reconstruction in L2 and H1-seminorm,
    pressure in L2 (zero mean when defined up to a constant), and the energy
    norm of I_h u - u_h in the scalar-per-component HHO seminorm."""
    mesh, geo = P.mesh, P.geo
    d, k = mesh.dim, P.k
    nT = dim_poly(d, k)
    lay = P.lays[0]
    UT, PT = recover(P, x)
    # pressure mean shift (exact p has zero mean on the unit box)
    if P.z[0] is not None:
        vol = np.array([cg.volume for cg in geo.cells])
        pm = sum(np.sqrt(v) * PT[c, 0] for c, v in enumerate(vol)) / vol.sum()
    else:
        pm = 0.0
    eu = eg = ep = ee = 0.0
    nu = ngu = npp = 0.0
    for c, L in enumerate(P.locs):
        xq, wq = L.qpts, L.qw
        phi = L.basis.values(xq)
        gphi = L.basis.grads(xq)
        Ud = x[face_dofs(mesh, c, d, lay.nF)].reshape(L.nfaces, d, L.nF)
        uq, guq = man.u(xq), man.grad_u(xq)
        # interpolate I_T u (L2 projections on the cell and the faces)
        vloc_I = np.zeros((d, L.nloc))
        vloc_h = np.zeros((d, L.nloc))
        for cc in range(d):
            vloc_I[cc, :nT] = np.einsum("q,q,qj->j", wq, uq[:, cc], phi[:, :nT])
            vloc_h[cc, :nT] = UT[c, cc * nT:(cc + 1) * nT]
            for i, f in enumerate(mesh.cell_faces(c)):
                xf, wf = geo.face_q[f]
                psi = geo.face_basis[f].values(xf)
                vloc_I[cc, nT + i * L.nF: nT + (i + 1) * L.nF] = np.einsum("q,q,qj->j", wf, man.u(xf)[:, cc], psi)
                vloc_h[cc, nT + i * L.nF: nT + (i + 1) * L.nF] = Ud[i, cc]
            ru = L.R @ vloc_h[cc]
            eu += np.dot(wq, (phi @ ru - uq[:, cc]) ** 2)
            eg += np.dot(wq, ((np.einsum("nid,i->nd", gphi, ru) - guq[:, cc, :]) ** 2).sum(axis=1))
            nu += np.dot(wq, uq[:, cc] ** 2)
            ngu += np.dot(wq, (guq[:, cc, :] ** 2).sum(axis=1))
            e = vloc_I[cc] - vloc_h[cc]
            ee += e @ L.a @ e
        ph = phi[:, :nT] @ PT[c] - pm
        pq = man.p(xq)
        ep += np.dot(wq, (ph - pq) ** 2)
        npp += np.dot(wq, pq ** 2)
    return {"u_L2": np.sqrt(eu), "grad_u_L2": np.sqrt(eg), "p_L2": np.sqrt(ep),
            "energy": np.sqrt(max(ee, 0.0)), "u_norm": np.sqrt(nu), "grad_norm": np.sqrt(ngu),
            "p_norm": np.sqrt(npp)}
