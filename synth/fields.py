"""Seeded problem data: body forces, boundary data and manufactured solutions.

These are inputs of the Stokes problem (Section 1, eq. stokesProb):
-Lap u + grad p = f, div u = 0, u = g_D on the Dirichlet part, and the traction
datum g_N on the Neumann part.  Throughout, g_N is read as the traction
(grad u - p I) n so that it enters the momentum residual with the sign used by
the HHO scheme of Section 2.3.1.

Every callable takes points ``x`` of shape [n, d] (and, for tractions, unit
normals ``nrm`` [n, d]) and returns an [n, d] (vector) or [n] (scalar) array.
"""
from __future__ import annotations

import os
from dataclasses import dataclass
from itertools import product
from typing import Callable, Optional
import numpy as np


@dataclass
class TrigSeries:
    """f_i(x) = sum_alpha a[i,alpha] prod_j cos(pi alpha_j x_j) + b[i,alpha] prod_j sin(pi alpha_j x_j),
    alpha ranging over {0..deg}^d."""
    dim: int
    alphas: np.ndarray      # [na, d] ints
    a: np.ndarray           # [d, na]
    b: np.ndarray           # [d, na]

    def __call__(self, x: np.ndarray) -> np.ndarray:
        x = np.atleast_2d(x)
        n, d = x.shape
        deg = int(self.alphas.max())
        m = deg + 1
        out = np.empty((n, self.a.shape[0]))
        # alphas enumerate the full tensor grid {0..deg}^d with alpha_0 slowest, so the
        # coefficients reshape to [out, m, ..., m] and the sum contracts one axis at a time
        A = self.a.reshape((-1,) + (m,) * d)
        B = self.b.reshape((-1,) + (m,) * d)

        def block(s0):
            th = np.pi * x[s0:s0 + (1 << 15)]                        # [p, d]
            # cos / sin of alpha * theta for alpha = 0..deg by the angle-addition recurrences
            ct = np.empty(th.shape + (m,))
            st = np.empty(th.shape + (m,))
            ct[..., 0], st[..., 0] = 1.0, 0.0
            if m > 1:
                c1, s1 = np.cos(th), np.sin(th)
                ct[..., 1], st[..., 1] = c1, s1
                for a in range(2, m):
                    ct[..., a] = 2.0 * c1 * ct[..., a - 1] - ct[..., a - 2]
                    st[..., a] = 2.0 * c1 * st[..., a - 1] - st[..., a - 2]
            ang = ct
            rc = np.tensordot(ct[:, d - 1], A, axes=([1], [A.ndim - 1]))   # [p, out, m, ..., m]
            rs = np.tensordot(st[:, d - 1], B, axes=([1], [B.ndim - 1]))
            for j in range(d - 2, -1, -1):
                shape = (ang.shape[0],) + (1,) * (rc.ndim - 2) + (m,)
                rc = (rc * ct[:, j].reshape(shape)).sum(axis=-1)
                rs = (rs * st[:, j].reshape(shape)).sum(axis=-1)
            out[s0:s0 + ang.shape[0]] = rc + rs

        starts = range(0, n, 1 << 15)                 # bounded temporaries, blocks on threads
        if n > (1 << 17):
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
                list(ex.map(block, starts))
        else:
            for s0 in starts:
                block(s0)
        return out


def trig_series(dim: int, seed: int, deg: int = 3) -> TrigSeries:
    """Random smooth body force: coefficients ~ N(0, 1/(1+|alpha|^2)) from
    ``numpy.random.default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    alphas = np.array(list(product(range(deg + 1), repeat=dim)), dtype=np.int64)
    sd = 1.0 / np.sqrt(1.0 + (alphas ** 2).sum(axis=1))
    a = rng.standard_normal((dim, len(alphas))) * sd
    b = rng.standard_normal((dim, len(alphas))) * sd
    return TrigSeries(dim, alphas, a, b)


def zero_field(dim: int) -> Callable[[np.ndarray], np.ndarray]:
    return lambda x: np.zeros((np.atleast_2d(x).shape[0], dim))


@dataclass
class Manufactured:
    """A Stokes solution (u, p) with f = -Lap u + grad p.  ``grad_u(x)`` returns
    [n, d, d] with grad_u[:, i, j] = d u_i / d x_j."""
    dim: int
    u: Callable
    p: Callable
    grad_u: Callable
    f: Callable
    name: str = ""
    p_mean_zero_on_unit_box: bool = True

    def traction(self, x: np.ndarray, nrm: np.ndarray) -> np.ndarray:
        G = self.grad_u(x)
        return np.einsum("nij,nj->ni", G, nrm) - self.p(x)[:, None] * nrm


def stokes_sincos_2d() -> Manufactured:
    """u = (sin(pi x) cos(pi y), -cos(pi x) sin(pi y)), p = x - y on the unit square."""
    pi = np.pi

    def u(x):
        return np.stack([np.sin(pi * x[:, 0]) * np.cos(pi * x[:, 1]),
                         -np.cos(pi * x[:, 0]) * np.sin(pi * x[:, 1])], axis=1)

    def p(x):
        return x[:, 0] - x[:, 1]

    def grad_u(x):
        sx, cx = np.sin(pi * x[:, 0]), np.cos(pi * x[:, 0])
        sy, cy = np.sin(pi * x[:, 1]), np.cos(pi * x[:, 1])
        G = np.empty((len(x), 2, 2))
        G[:, 0, 0] = pi * cx * cy
        G[:, 0, 1] = -pi * sx * sy
        G[:, 1, 0] = pi * sx * sy
        G[:, 1, 1] = -pi * cx * cy
        return G

    def f(x):
        sx, cx = np.sin(pi * x[:, 0]), np.cos(pi * x[:, 0])
        sy, cy = np.sin(pi * x[:, 1]), np.cos(pi * x[:, 1])
        return np.stack([2 * pi ** 2 * sx * cy + 1.0, -2 * pi ** 2 * cx * sy - 1.0], axis=1)

    return Manufactured(2, u, p, grad_u, f, name="sincos2d")


# ---------------------------------------------------------------- polynomials
def _monomials(dim, deg):
    return [a for a in product(range(deg + 1), repeat=dim) if sum(a) <= deg]


class _Poly:
    """Dense multivariate polynomial sum_c coef[c] x^alpha_c (input generation only)."""

    def __init__(self, dim, terms):
        self.dim = dim
        self.terms = {tuple(a): float(c) for a, c in terms.items() if c != 0.0}

    def __call__(self, x):
        x = np.atleast_2d(x)
        out = np.zeros(len(x))
        for a, c in self.terms.items():
            out += c * np.prod(x ** np.array(a)[None, :], axis=1)
        return out

    def d(self, j):
        t = {}
        for a, c in self.terms.items():
            if a[j] > 0:
                b = list(a)
                b[j] -= 1
                t[tuple(b)] = t.get(tuple(b), 0.0) + c * a[j]
        return _Poly(self.dim, t)

    def __add__(self, o):
        t = dict(self.terms)
        for a, c in o.terms.items():
            t[a] = t.get(a, 0.0) + c
        return _Poly(self.dim, t)

    def scale(self, s):
        return _Poly(self.dim, {a: s * c for a, c in self.terms.items()})

    def box_mean(self):
        # mean over the unit box [0,1]^d
        return sum(c * np.prod([1.0 / (ai + 1) for ai in a]) for a, c in self.terms.items())


def polynomial_stokes(dim: int, k: int, seed: int = 0) -> Manufactured:
    """Seeded divergence-free u in P^{k+1}(R^d)^d and p in P^k with zero mean on
    the unit box.  u is the curl of a random polynomial stream function
    (d=2: scalar psi in P^{k+2}; d=3: vector potential in P^{k+2}^3)."""
    rng = np.random.default_rng(seed)
    if dim == 2:
        psi = _Poly(2, {a: rng.standard_normal() for a in _monomials(2, k + 2)})
        comps = [psi.d(1), psi.d(0).scale(-1.0)]
    else:
        A = [_Poly(3, {a: rng.standard_normal() for a in _monomials(3, k + 2)}) for _ in range(3)]
        comps = [A[2].d(1) + A[1].d(2).scale(-1.0),
                 A[0].d(2) + A[2].d(0).scale(-1.0),
                 A[1].d(0) + A[0].d(1).scale(-1.0)]
    pp = _Poly(dim, {a: rng.standard_normal() for a in _monomials(dim, k)})
    pp = pp + _Poly(dim, {(0,) * dim: -pp.box_mean()})
    grads = [[c.d(j) for j in range(dim)] for c in comps]
    lap = [sum((g[j].d(j) for j in range(1, dim)), g[0].d(0)) for g in grads]
    dp = [pp.d(j) for j in range(dim)]
    fcomp = [lap[i].scale(-1.0) + dp[i] for i in range(dim)]

    def u(x):
        return np.stack([c(x) for c in comps], axis=1)

    def p(x):
        return pp(x)

    def grad_u(x):
        return np.stack([np.stack([g[j](x) for j in range(dim)], axis=1) for g in grads], axis=1)

    def f(x):
        return np.stack([c(x) for c in fcomp], axis=1)

    return Manufactured(dim, u, p, grad_u, f, name=f"poly{dim}d_k{k}_s{seed}")


def problem_data(man: Optional[Manufactured], forcing: Optional[TrigSeries], dim: int):
    """(f, g_D, g_N) callables: from a manufactured solution, or a body force with
    homogeneous boundary data."""
    if man is not None:
        return man.f, man.u, man.traction
    z = zero_field(dim)
    return forcing, z, (lambda x, n: z(x))
