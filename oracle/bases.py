"""Hierarchical L2-orthonormal bases (test infrastructure; see the package header).

Section 4.2 uses hierarchical orthonormal bases so that the restriction from
P^{k_l}(X) to P^{k_{l+1}}(X) is a unit-diagonal rectangular matrix (sub-block
extraction).  The bases here are obtained by Gram-Schmidt (modified, applied
twice) in L2(X) of scaled monomials listed by total degree, then
lexicographically with the first exponent decreasing:

* cell T:  ((x - x_T)/h_T)^alpha, |alpha| <= k+1;
* face F:  (xi_1, .., xi_{d-1})^beta with xi_i = (x - x_F).t_i / h_F.

Because degree-graded Gram-Schmidt never mixes a higher degree into a lower
one, the first dim P^l functions span P^l for every l, and the first cell
function is |T|^{-1/2} (the mean-first pressure basis of Section 4.1.2).
"""
from __future__ import annotations

from math import comb
import numpy as np


def exponents(dim: int, deg: int):
    """Exponents of the monomials of total degree <= deg in the graded order."""
    out = []
    for n in range(deg + 1):
        if dim == 1:
            out.append((n,))
        elif dim == 2:
            for a in range(n, -1, -1):
                out.append((a, n - a))
        else:
            for a in range(n, -1, -1):
                for b in range(n - a, -1, -1):
                    out.append((a, b, n - a - b))
    return np.array(out, dtype=np.int64)


def dim_poly(dim: int, deg: int) -> int:
    return comb(deg + dim, dim) if deg >= 0 else 0


def monomials(xi: np.ndarray, E: np.ndarray):
    """Values [n, N] of xi^E (xi [n, dim])."""
    return np.prod(xi[:, None, :] ** E[None, :, :], axis=2)


def monomial_grads(xi: np.ndarray, E: np.ndarray, scale: float):
    """Gradients [n, N, dim] w.r.t. x of (xi)^E where xi = (x - x0)/scale."""
    n, dim = xi.shape
    G = np.zeros((n, len(E), dim))
    for j in range(dim):
        Ej = E.copy()
        Ej[:, j] = np.maximum(E[:, j] - 1, 0)
        G[:, :, j] = E[None, :, j] * monomials(xi, Ej) / scale
    return G


def gram_schmidt(M: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Coefficients C [N, N] with phi_i = sum_j C[i, j] m_j orthonormal in the
    discrete inner product sum_q w_q m(x_q) m(x_q).  Modified Gram-Schmidt,
    each vector orthogonalised twice."""
    N = M.shape[1]
    C = np.zeros((N, N))
    V = np.zeros_like(M)
    for i in range(N):
        c = np.zeros(N)
        c[i] = 1.0
        v = M[:, i].copy()
        for _ in range(2):
            for j in range(i):
                r = np.dot(w, v * V[:, j])
                v -= r * V[:, j]
                c -= r * C[j]
        nv = np.sqrt(np.dot(w, v * v))
        V[:, i] = v / nv
        C[i] = c / nv
    return C


class CellBasis:
    """Orthonormal hierarchical basis of P^{deg}(T)."""

    def __init__(self, centroid, diam, qpts, qw, deg: int):
        self.x0, self.h, self.deg = centroid, diam, deg
        self.E = exponents(len(centroid), deg)
        self.C = gram_schmidt(monomials(self._xi(qpts), self.E), qw)

    def _xi(self, x):
        return (x - self.x0[None, :]) / self.h

    def values(self, x):
        return monomials(self._xi(x), self.E) @ self.C.T

    def grads(self, x):
        G = monomial_grads(self._xi(x), self.E, self.h)
        return np.einsum("nmd,im->nid", G, self.C)


class FaceBasis:
    """Orthonormal hierarchical basis of P^{deg}(F) in the face's tangent frame."""

    def __init__(self, fgeo, qpts, qw, deg: int):
        self.x0, self.h, self.t, self.deg = fgeo.centroid, fgeo.diam, fgeo.tangents, deg
        self.E = exponents(self.t.shape[0], deg)
        self.C = gram_schmidt(monomials(self._xi(qpts), self.E), qw)

    def _xi(self, x):
        return ((x - self.x0[None, :]) @ self.t.T) / self.h

    def values(self, x):
        return monomials(self._xi(x), self.E) @ self.C.T
