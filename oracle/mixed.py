"""Single-precision emulation of the V-cycle (test infrastructure; see the package
header).  Not in the paper.

The mixed-precision solver keeps the outer flexible GMRES, the local
factorisations and the coarsest-level solve in FP64 and runs the levels above
the coarsest in FP32: their operators and smoother preconditioners are the FP64
ones rounded to float32, and every vector operation on them is done in float32.
This module replays that with NumPy float32 arithmetic:

* level matrices S_l (l < L) and the Schwarz patch inverses and weights are
  rounded to float32 once;
* residuals, preconditioner applications, matrix-vector products and the
  smoother's iterate are float32 arrays, combined in float32;
* the smoother's small least-squares problem (at most 3 x 2) is solved in
  float64 from float32 dot products, and its coefficients are rounded to
  float32 before they scale float32 vectors;
* the defect is restricted in float32, rounded up to float64 for the coarsest
  solve (FP64, the Hierarchy's own), and the coarse correction is rounded to
  float32 before it is added.

The V-cycle's steps are those of ``oracle.multilevel.Hierarchy.vcycle``.

``product_copy_block`` gives a cell's face block of the V-cycle copy formed by
the matrix-core product (not in the paper): the elimination of eq. ST.1 (and
ST.2) in factored form, Cholesky factor L of the cell block A_TT, W = L^{-1} A_Td,
and for v&p-cond Y = L^{-1} B_T^T, C = B_d^T - W^T Y, Sigma = the non-mean block
of Y^T Y with Cholesky factor L_s and Z = L_s^{-1} C~^T; the factors are rounded
to bfloat16 and the face block is A_dd (rounded to float32) - W^T W (+ Z^T Z for
v&p-cond), here with exact products and sums of the rounded values.

``round_bf16`` gives the bfloat16 storage of the 16-bit mode: a bfloat16 number
is an IEEE binary32 number whose 16 low significand bits are zero, and a float32
value is stored as the nearest such number, ties to the one whose lowest kept
bit is zero (round to nearest even); values keep float32 arithmetic after that.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def round_bf16(a):
    """Nearest bfloat16 numbers (ties to even) of the float32 values of ``a``,
    as float32.  Written from the definition: the two bfloat16 neighbours of x
    are x with its 16 low bits cleared (towards zero) and the next bfloat16 away
    from zero; the nearer wins, an exact tie goes to the one with an even kept
    significand.  NaN and infinities are left as they are."""
    x = np.asarray(a, dtype=F32)
    bits = x.view(np.uint32)
    lo = bits & np.uint32(0xFFFF0000)                       # truncated towards zero
    hi = (lo.astype(np.uint64) + 0x10000).astype(np.uint32)  # next one away from zero
    rest = bits & np.uint32(0xFFFF)                          # distance to lo in units of 2^-16 ulp
    up = (rest > 0x8000) | ((rest == 0x8000) & ((lo >> 16) & 1 == 1))
    out = np.where(up, hi, lo).astype(np.uint32).view(F32)
    return np.where(np.isfinite(x), out, x).astype(F32)


class Schwarz32:
    """A cell-patch Schwarz preconditioner with float32 values."""

    def __init__(self, M):
        self.N = M.N
        self.patches = M.patches
        self.weights = [w.astype(F32) for w in M.weights]
        self.inv = [Ai.astype(F32) for Ai in M.inv]

    def __call__(self, r):
        assert r.dtype == F32
        z = np.zeros(self.N, dtype=F32)
        for idx, w, Ai in zip(self.patches, self.weights, self.inv):
            z[idx] += w * (Ai @ r[idx])
        return z


def _gmres_steps32(S, M, w, r0, m):
    """m right-preconditioned GMRES iterations from w (float32 vectors), CGS2."""
    beta = np.float64(np.linalg.norm(r0.astype(np.float64)))
    if beta == 0.0:
        return w.copy()
    V, Z = [(r0 / F32(beta)).astype(F32)], []
    H = np.zeros((m + 1, m))
    n = 0
    for j in range(m):
        z = M(V[j])
        Z.append(z)
        u = S @ z
        h = np.zeros(j + 1)
        for _ in range(2):
            hh = np.array([np.float64(np.dot(v, u)) for v in V])
            for hi, v in zip(hh, V):
                u = u - F32(hi) * v
            h += hh
        H[:j + 1, j] = h
        H[j + 1, j] = np.linalg.norm(u.astype(np.float64))
        n = j + 1
        if H[j + 1, j] <= 1e-7 * beta:
            break
        V.append((u / F32(H[j + 1, j])).astype(F32))
    e1 = np.zeros(n + 1)
    e1[0] = beta
    y = np.linalg.lstsq(H[:n + 1, :n], e1, rcond=None)[0]
    out = w.copy()
    for yi, zi in zip(y, Z):
        out = out + F32(yi) * zi
    return out


class Vcycle32:
    """MG_V(0, b, 0) with every level above the coarsest in float32."""

    def __init__(self, H):
        self.H = H
        self.S = [S.astype(F32).tocsr() for S in H.S[:-1]]
        self.prec = [Schwarz32(M) for M in H.prec[:-1]]

    def _v(self, l, b):
        H = self.H
        S = self.S[l]
        w = np.zeros_like(b)
        w = _gmres_steps32(S, self.prec[l], w, b - S @ w, H.smooth_its)      # pre-smoothing
        d = (b - S @ w)[H.idx[l]]                                           # restricted defect
        if l + 1 == H.L:
            c = H.coarse_solve(d.astype(np.float64)).astype(F32)
        else:
            c = self._v(l + 1, d)
        w = w.copy()
        w[H.idx[l]] += c                                                    # coarse correction
        return _gmres_steps32(S, self.prec[l], w, b - S @ w, H.smooth_its)  # post-smoothing

    def __call__(self, b):
        return self._v(0, np.asarray(b).astype(F32)).astype(np.float64)


def product_copy_block(L, cond):
    """(block, bound): the face block of one cell's Schur complement as the
    matrix-core product forms it (see the module header), in the vector unknown
    order (face, component, mode), and |left| |right| summed over the product,
    the scale of its single-precision accumulation error."""
    from scipy.linalg import solve_triangular
    from .hho import vector_system
    A_TT, A_Td, A_dd, B_T, B_d, _, _, _ = vector_system(L)
    Lc = np.linalg.cholesky(A_TT)
    W = solve_triangular(Lc, A_Td, lower=True)
    Wb = round_bf16(W.astype(F32)).astype(np.float64)
    base = A_dd.astype(F32).astype(np.float64)
    block = base - Wb.T @ Wb
    bound = np.abs(Wb).T @ np.abs(Wb)
    if cond == "vp":
        Y = solve_triangular(Lc, B_T.T, lower=True)          # [d nT, nT]
        C = B_d.T - W.T @ Y                                 # [d m, nT]
        Sg = Y[:, 1:].T @ Y[:, 1:]
        Ls = np.linalg.cholesky(Sg)
        Z = solve_triangular(Ls, C[:, 1:].T, lower=True)     # [nT - 1, d m]
        Zb = round_bf16(Z.astype(F32)).astype(np.float64)
        block = block + Zb.T @ Zb
        bound = bound + np.abs(Zb).T @ np.abs(Zb)
    return block, bound

