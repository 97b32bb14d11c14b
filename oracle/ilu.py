"""Zero-fill incomplete LU factorisation, the preconditioner of the paper's
smoother (test infrastructure; see the package header).

Section 3.3 smooths with a few GMRES iterations preconditioned by ILU, and the
multilevel solver options of Section 5.2 fix two such iterations.  The paper
names no fill level or ordering; the readings here are the usual defaults of
its software: fill level 0 and the natural ordering of the global unknowns
(faces, then cells, in the global layout).

Pattern.  The condensed operator couples two unknowns when they belong to a
common cell, and the assembled matrix stores exactly those positions (every
cell contributes its whole dense condensed block, zero entries included), so
the factor pattern is that structural cell-stencil pattern of the level matrix.

Algorithm (row-wise elimination restricted to the pattern): for every row i in
increasing order and every k < i with (i, k) in the pattern, in increasing k,
the multiplier l_ik = a_ik / u_kk is formed and row k's upper part is
subtracted from row i at the positions (i, j), j > k, that the pattern holds;
entries outside the pattern are dropped.  The result satisfies (L U)_ij = a_ij
on the pattern, L unit lower triangular and U upper triangular.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class ILU0:
    def __init__(self, A: sp.spmatrix):
        A = sp.csr_matrix(A, dtype=np.float64, copy=True)
        A.sort_indices()
        n = A.shape[0]
        ptr, col, val = A.indptr, A.indices, A.data
        # position of each (i, j) of the pattern, per row
        pos = [dict(zip(col[ptr[i]:ptr[i + 1]].tolist(), range(ptr[i], ptr[i + 1]))) for i in range(n)]
        diag = np.empty(n, dtype=np.int64)
        for i in range(n):
            if i not in pos[i]:
                raise ValueError(f"ILU(0): row {i} has no diagonal entry")
            diag[i] = pos[i][i]
        for i in range(n):
            row = pos[i]
            for e in range(ptr[i], ptr[i + 1]):
                k = col[e]
                if k >= i:
                    break
                val[e] /= val[diag[k]]               # l_ik
                lik = val[e]
                for e2 in range(diag[k] + 1, ptr[k + 1]):   # u_kj, j > k
                    j = col[e2]
                    q = row.get(j)
                    if q is not None:
                        val[q] -= lik * val[e2]
            if val[diag[i]] == 0.0:
                raise ZeroDivisionError(f"ILU(0): zero pivot in row {i}")
        self.n = n
        self.F = A
        self.L = (sp.tril(A, k=-1) + sp.eye(n)).tocsr()
        self.U = sp.triu(A).tocsr()

    def __call__(self, r: np.ndarray) -> np.ndarray:
        """z = U^{-1} L^{-1} r."""
        y = spla.spsolve_triangular(self.L, r, lower=True, unit_diagonal=True)
        return spla.spsolve_triangular(self.U, y, lower=False)
