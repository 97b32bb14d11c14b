"""Coarsest-level solver of the GPU library, replayed on the CPU (test
infrastructure; see the package header).

The paper solves the coarsest level with a sparse LU (2D) or ILU-GMRES to a
three-orders-of-magnitude residual reduction (3D), Section 5.2.2.  The GPU
library keeps the "GMRES to 1e-3" rule but preconditions it with a
block-triangular Stokes preconditioner whose velocity block is approximated by
one smoothed-aggregation AMG V-cycle.  This module is the plain definition of
that preconditioner, used to check the GPU implementation:

* scalar face operator  s[f,g] = (1/d) sum_c S[(f,c),(g,c)]   (coarsest level, k_L = 0)
* aggregation: nodes in index order; an unaggregated node opens an aggregate
  holding itself and its unaggregated neighbours in the aggregation graph G
  (G_0 = pattern of A_0, G_{l+1} = pattern of T^T G_l T: aggregates are
  neighbours when their members are)
* lambda: 15 power-iteration steps v <- D^{-1} A v / |.| from the start vector
  v_i = frac(i * 2654435761 / 2^32) - 1/2, times 1.05 (estimate of rho(D^{-1} A))
* tentative prolongator T (0/1), P = (I - (omega/lambda) D^{-1} A)^s T with
  omega = 4/3 and s prolongator smoothing steps: the most, up to 1 (the
  default) or 2 (on request), for which A_next = P^T A P holds at most 160 entries
  per row (structurally); down to <= 128 unknowns, then a dense inverse; when no
  s >= 1 keeps A_next that sparse coarsening stops, and such a coarsest level
  gets 6 damped-Jacobi sweeps from zero
* V-cycle with nu (default 2) damped-Jacobi sweeps of weight 4/(3 lambda) before
  and after the coarse correction
* pressure Schur approximation  S_T = sum_{(f,c)} C[(f,c),T]^2 / S[(f,c),(f,c)]
* apply: y = -g / S_T,   x = V-cycle(f - C y) per velocity component.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

OMEGA_SA = 4.0 / 3.0
COARSEST = 128
MAX_ROW_NNZ = 160
COARSE_SWEEPS = 6
POWER_STEPS = 15
LAMBDA_SAFETY = 1.05


def start_vector(n: int) -> np.ndarray:
    """Deterministic start vector of the power iteration (Knuth multiplicative hash)."""
    i = np.arange(n, dtype=np.uint64)
    h = (i * np.uint64(2654435761)) % np.uint64(2 ** 32)
    return h.astype(np.float64) / 2.0 ** 32 - 0.5


def spectral_radius_estimate(A: sp.csr_matrix) -> float:
    Di = 1.0 / A.diagonal()
    v = start_vector(A.shape[0])
    lam = 1.0
    for _ in range(POWER_STEPS):
        v = Di * (A @ v)
        lam = float(np.linalg.norm(v))
        v = v / lam
    return LAMBDA_SAFETY * lam


def aggregate(A: sp.csr_matrix) -> np.ndarray:
    n = A.shape[0]
    agg = -np.ones(n, dtype=np.int64)
    na = 0
    for i in range(n):
        if agg[i] >= 0:
            continue
        for j in A.indices[A.indptr[i]:A.indptr[i + 1]]:
            if agg[j] < 0:
                agg[j] = na
        agg[i] = na
        na += 1
    return agg


class SA:
    def __init__(self, A: sp.csr_matrix, nu: int = 2, p_steps: int = 1):
        self.nu = nu
        self.p_steps = p_steps
        self.steps = []   # smoothing steps taken per level
        self.levels = []
        self.lams = []
        A = sp.csr_matrix(A)
        A.sort_indices()
        G = A.copy()
        G.data[:] = 1.0
        while A.shape[0] > COARSEST:
            agg = aggregate(G)
            na = int(agg.max()) + 1
            if na >= A.shape[0]:
                break
            T = sp.csr_matrix((np.ones(A.shape[0]), (np.arange(A.shape[0]), agg)), shape=(A.shape[0], na))
            # smoothing steps of this level: the most (<= p_steps) whose next operator
            # stays below the density bound (structurally; P pattern: T, then P + A P
            # per step); none fits: this level is the coarsest
            Ab = A.copy()
            Ab.data[:] = 1.0
            steps = 0
            for st in range(p_steps, 0, -1):
                Pb = T.copy()
                for _ in range(st):
                    Pb = (Pb + Ab @ Pb).tocsr()
                    Pb.data[:] = 1.0
                if (Pb.T @ Ab @ Pb).nnz <= MAX_ROW_NNZ * na:
                    steps = st
                    break
            if steps == 0:
                break
            D = A.diagonal()
            lam = spectral_radius_estimate(A)
            P = T
            for _ in range(steps):
                P = (P - (OMEGA_SA / lam) * (sp.diags(1.0 / D) @ (A @ P))).tocsr()
            self.steps.append(steps)
            self.levels.append((A, P, 1.0 / D))
            self.lams.append(lam)
            A = (P.T @ A @ P).tocsr()
            A.sort_indices()
            G = (T.T @ G @ T).tocsr()
            G.data[:] = 1.0
            G.sort_indices()
        self.Ac = A
        if A.shape[0] <= COARSEST:
            self.Ainv = np.linalg.inv(A.toarray())
        else:
            self.Ainv = None
            self.Dc = 1.0 / A.diagonal()
            self.lam_c = spectral_radius_estimate(A)
        self.sizes = [L[0].shape[0] for L in self.levels] + [A.shape[0]]

    def vcycle(self, r: np.ndarray, l: int = 0) -> np.ndarray:
        if l == len(self.levels):
            if self.Ainv is not None:
                return self.Ainv @ r
            w = 4.0 / (3.0 * self.lam_c)
            x = np.zeros_like(r)
            for _ in range(COARSE_SWEEPS):
                x = x + w * self.Dc * (r - self.Ac @ x)
            return x
        A, P, Di = self.levels[l]
        w = 4.0 / (3.0 * self.lams[l])
        x = np.zeros_like(r)
        for _ in range(self.nu):
            x = x + w * Di * (r - A @ x)
        x = x + P @ self.vcycle(P.T @ (r - A @ x), l + 1)
        for _ in range(self.nu):
            x = x + w * Di * (r - A @ x)
        return x


class BlockStokesPrec:
    """Block-triangular preconditioner of the coarsest (k = 0) level."""

    def __init__(self, S: sp.csr_matrix, nface_dofs: int, d: int, nu: int = 2, p_steps: int = 1):
        S = sp.csr_matrix(S)
        self.nf, self.d = nface_dofs, d
        nfaces = nface_dofs // d
        blocks = [S[c:nface_dofs:d][:, c:nface_dofs:d] for c in range(d)]
        s = sum(blocks[1:], blocks[0]) / d
        self.amg = SA(s.tocsr(), nu, p_steps)
        C = S[:nface_dofs, nface_dofs:].tocsc()
        diagA = S.diagonal()[:nface_dofs]
        Sd = np.asarray((C.multiply(C)).T @ (1.0 / diagA)).ravel()
        Sd[~(Sd > 0)] = 1.0
        self.Sd = Sd
        self.C = C.tocsr()
        del nfaces

    def __call__(self, v: np.ndarray) -> np.ndarray:
        f, g = v[:self.nf], v[self.nf:]
        y = -g / self.Sd
        rhs = (f - self.C @ y).reshape(-1, self.d)
        x = np.stack([self.amg.vcycle(rhs[:, c]) for c in range(self.d)], axis=1).ravel()
        return np.concatenate([x, y])
