"""p-multilevel V-cycle of Section 3.3 (test infrastructure; see package header).

Smoother preconditioner.  The paper preconditions its smoothing GMRES
iterations with ILU; ``oracle.ilu.ILU0`` is that preconditioner (zero fill,
natural ordering) and ``oracle.solve.hierarchy(smoother="ilu")`` selects it.
The GPU library's default replaces ILU by a cell-patch additive Schwarz
preconditioner, and this module replays that choice exactly:
for every cell T the patch holds the unknowns of the faces of T and the
pressure unknowns of T at the current level; the patch matrix is the global
level matrix restricted to the patch; the correction of the patch is solved
densely and added back with weight 1/card(T_F) on face unknowns (1/2 on interior
faces) and 1 on pressure unknowns.

Coarsest level: either a direct solve (bordered with the constant-pressure
vector when the operator is singular), or GMRES to a relative tolerance
(Section 5.2.2 uses LU in 2D and ILU-GMRES to 1e-3 in 3D) preconditioned by the
same Schwarz method ("gmres") or by the block-triangular preconditioner with a
smoothed-aggregation velocity block of ``oracle.amg`` ("amg", k_L = 0 only).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .krylov import gmres_steps, gmres_solve
from .system import face_dofs


class Schwarz:
    def __init__(self, S: sp.csr_matrix, mesh, lay):
        d, nF, nP = lay.d, lay.nF, lay.nP
        fc = mesh.face_cells()
        nTF = (fc >= 0).sum(axis=1)
        self.patches, self.weights, self.inv = [], [], []
        Sd = S.tocsr()
        for c in range(mesh.n_cells):
            fd = face_dofs(mesh, c, d, nF)
            idx = np.concatenate([fd, lay.off + c * nP + np.arange(nP)])
            wf = np.repeat(1.0 / nTF[mesh.cell_faces(c)], d * nF)
            self.patches.append(idx)
            self.weights.append(np.concatenate([wf, np.ones(nP)]))
            self.inv.append(np.linalg.inv(Sd[idx][:, idx].toarray()))
        self.N = S.shape[0]

    def __call__(self, r):
        z = np.zeros(self.N)
        for idx, w, Ai in zip(self.patches, self.weights, self.inv):
            z[idx] += w * (Ai @ r[idx])
        return z


@dataclass
class Hierarchy:
    S: list                 # level matrices (csr), level 0 finest
    idx: list               # idx[l]: level-l index of each level-(l+1) unknown
    prec: list              # Schwarz per level (the coarsest too, for GMRES)
    z: list                 # constant-pressure vector per level or None
    smooth_its: int = 2
    coarse: str = "direct"  # "direct" | "gmres" | "amg"
    coarse_rtol: float = 1e-3
    coarse_restart: int = 30
    coarse_maxit: int = 500
    coarse_its: list = field(default_factory=list)
    nface_dofs: list = field(default_factory=list)
    dim: int = 2
    amg_nu: int = 2
    learned: object = None  # optional r -> correction on level 0 (oracle.mlp.apply), see smooth()
    _lu: object = None
    _amg: object = None

    @property
    def L(self):
        return len(self.S) - 1

    def restrict(self, l, v):
        return v[self.idx[l]]

    def prolong(self, l, c):
        out = np.zeros(self.S[l].shape[0])
        out[self.idx[l]] = c
        return out

    def coarse_solve(self, d):
        L = self.L
        S = self.S[L]
        z = self.z[L]
        if self.coarse == "direct":
            if self._lu is None:
                if z is not None:
                    Sb = sp.bmat([[S, sp.csr_matrix(z[:, None])], [sp.csr_matrix(z[None, :]), None]]).tocsc()
                else:
                    Sb = S.tocsc()
                self._lu = spla.splu(Sb)
            rhs = np.concatenate([d, [0.0]]) if z is not None else d
            return self._lu.solve(rhs)[:S.shape[0]]
        M = self.prec[L]
        if self.coarse == "amg":
            if self._amg is None:
                from .amg import BlockStokesPrec
                self._amg = BlockStokesPrec(S, self.nface_dofs[L], self.dim, self.amg_nu)
            M = self._amg
        x, its = gmres_solve(lambda v: S @ v, M, d, self.coarse_rtol, self.coarse_restart, self.coarse_maxit)
        self.coarse_its.append(its)
        return x

    def smooth(self, l, b, w):
        """One smoothing step: right-preconditioned GMRES(smooth_its); on level 0
        with a learned correction N, the residual is minimised over
        span{M r, M A M r, N(r)} instead (not in the paper)."""
        S = self.S[l]
        A = lambda v: S @ v  # noqa: E731
        r = b - S @ w
        if l == 0 and self.learned is not None:
            from .mlp import mr_step
            M = self.prec[l]
            dirs = [M(r)]
            if self.smooth_its == 2:
                dirs.append(M(S @ dirs[0]))
            dirs.append(self.learned(r))
            return mr_step(A, dirs, w, r)
        return gmres_steps(A, self.prec[l], w, r, self.smooth_its)

    def vcycle(self, l, b, w=None):
        """MG_V(l, b, w) of the algorithm in Section 3.3.  On the coarsest level the
        algorithm solves (so a one-level hierarchy is its coarsest solve)."""
        if l == self.L:
            return self.coarse_solve(b)
        S = self.S[l]
        w = np.zeros_like(b) if w is None else w
        w = self.smooth(l, b, w)                                           # pre-smoothing
        dc = self.restrict(l, b - S @ w)                                   # restricted defect
        if l + 1 == self.L:
            c = self.coarse_solve(dc)
        else:
            c = self.vcycle(l + 1, dc, None)
        w = w + self.prolong(l, c)                                         # coarse correction
        w = self.smooth(l, b, w)                                           # post-smoothing
        return w
