"""Pins of the oracle's quadrature, bases and local HHO operators against closed
forms (Sections 2.1-2.2, 4.2).  CPU only."""
import numpy as np
import pytest

from synth import cartesian_quads, voronoi_lloyd, cartesian_hexes
from oracle import quadrature as Q
from oracle.bases import dim_poly, exponents
from oracle.hho import mesh_geometry, local_hho, vector_system
from oracle.geometry import cell_quadrature


def _zero(d):
    z = lambda x: np.zeros((len(x), d))  # noqa: E731
    return z, z, (lambda x, n: z(x))


def test_quadrature_exact_monomials():
    # integral of x^a y^b over the unit triangle (0,0),(1,0),(0,1) = a! b! / (a+b+2)!
    from math import factorial
    v0, v1, v2 = np.array([0., 0.]), np.array([1., 0.]), np.array([0., 1.])
    for deg in range(0, 13):
        p, w = Q.triangle(v0, v1, v2, deg)
        for a in range(deg + 1):
            b = deg - a
            exact = factorial(a) * factorial(b) / factorial(a + b + 2)
            assert abs(np.dot(w, p[:, 0] ** a * p[:, 1] ** b) - exact) < 1e-15
    # box [0,2]x[0,1]x[0,3]: x^a y^b z^c
    lo, hi = np.zeros(3), np.array([2., 1., 3.])
    p, w = Q.box(lo, hi, 9)
    for a, b, c in [(0, 0, 0), (3, 2, 4), (9, 0, 0), (1, 4, 4)]:
        exact = 2 ** (a + 1) / (a + 1) / (b + 1) * 3 ** (c + 1) / (c + 1)
        assert abs(np.dot(w, p[:, 0] ** a * p[:, 1] ** b * p[:, 2] ** c) - exact) < 1e-11 * exact
    # tetrahedron: int x^a y^b z^c over the unit simplex = a!b!c!/(a+b+c+3)!
    p, w = Q.tetra(np.zeros(3), np.array([1., 0, 0]), np.array([0, 1., 0]), np.array([0, 0, 1.]), 8)
    for a, b, c in [(0, 0, 0), (2, 3, 3), (8, 0, 0), (1, 1, 1)]:
        exact = factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)
        assert abs(np.dot(w, p[:, 0] ** a * p[:, 1] ** b * p[:, 2] ** c) - exact) < 1e-15


def test_polygon_area_and_dims():
    ring = np.array([[0, 0], [2, 0], [3, 1], [1, 2], [-0.5, 1]], dtype=float)
    p, w = Q.polygon(ring, 4)
    x, y = ring[:, 0], ring[:, 1]
    area = 0.5 * abs(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))
    assert abs(w.sum() - area) < 1e-14
    assert [dim_poly(2, k) for k in range(4)] == [1, 3, 6, 10]
    assert [dim_poly(3, k) for k in range(4)] == [1, 4, 10, 20]
    assert len(exponents(3, 3)) == 20 and len(exponents(2, 4)) == 15


@pytest.mark.parametrize("mesh,k", [(cartesian_quads(3), 2), (voronoi_lloyd(10, 3), 3), (cartesian_hexes(2), 1)])
def test_bases_orthonormal_hierarchical(mesh, k):
    geo = mesh_geometry(mesh, k)
    L = local_hho(mesh, geo, 0, 50.0, *_zero(mesh.dim))
    phi = L.basis.values(L.qpts)
    G = phi.T @ (L.qw[:, None] * phi)
    assert np.abs(G - np.eye(len(G))).max() < 1e-13
    # mean-first: phi_0 = |T|^{-1/2}, all other functions have zero mean
    vol = geo.cells[0].volume
    assert np.allclose(phi[:, 0], vol ** -0.5, rtol=1e-13)
    assert np.abs(L.qw @ phi[:, 1:]).max() < 1e-13
    # hierarchy: every monomial of degree l is reproduced by the first dim P^l functions
    x0, h = geo.cells[0].centroid, geo.cells[0].diam
    for l in range(k + 2):
        n = dim_poly(mesh.dim, l)
        for e in exponents(mesh.dim, l)[-3:]:
            mvals = np.prod(((L.qpts - x0) / h) ** e[None, :], axis=1)
            coef = (L.qw * mvals) @ phi[:, :n]
            assert np.abs(phi[:, :n] @ coef - mvals).max() < 1e-12
    for f in mesh.cell_faces(0):
        xf, wf = geo.face_q[f]
        psi = geo.face_basis[f].values(xf)
        assert np.abs(psi.T @ (wf[:, None] * psi) - np.eye(psi.shape[1])).max() < 1e-13


def _interp(mesh, geo, L, c, w):
    nT = L.nT
    v = np.zeros(L.nloc)
    v[:nT] = (L.qw * w(L.qpts)) @ L.basis.values(L.qpts)[:, :nT]
    for i, f in enumerate(mesh.cell_faces(c)):
        xf, wf = geo.face_q[f]
        v[nT + i * L.nF: nT + (i + 1) * L.nF] = (wf * w(xf)) @ geo.face_basis[f].values(xf)
    return v


@pytest.mark.parametrize("mesh,k", [(cartesian_quads(4), 1), (voronoi_lloyd(25, 5), 3),
                                    (cartesian_hexes(3), 2)])
def test_reconstruction_and_stabilisation_exact(mesh, k):
    """P_T I_T w = w and r_TF(I_T w) = 0 for w in P^{k+1}(T) (Section 2.2), so on an
    interior cell a_T(I w, I w) = |grad w|^2_T."""
    geo = mesh_geometry(mesh, k)
    c = next(c for c in range(mesh.n_cells) if all(mesh.face_bc[mesh.cell_faces(c)] == 0))
    L = local_hho(mesh, geo, c, 50.0, *_zero(mesh.dim))
    rng = np.random.default_rng(1)
    coef = rng.standard_normal(dim_poly(mesh.dim, k + 1))
    w = lambda x: L.basis.values(x) @ coef  # noqa: E731
    v = _interp(mesh, geo, L, c, w)
    assert np.abs(L.R @ v - coef).max() < 1e-12 * np.abs(coef).max()
    gw = np.einsum("nid,i->nd", L.basis.grads(L.qpts), coef)
    exact = L.qw @ (gw ** 2).sum(1)
    assert abs(v @ L.a @ v - exact) < 1e-11 * exact
    # discrete divergence: (B I w_vec, q) = -(div w, q)_T on an interior cell
    for cc in range(mesh.dim):
        lhs = L.B[cc] @ v
        rhs = -(L.qw * gw[:, cc]) @ L.basis.values(L.qpts)[:, :L.nT]
        assert np.abs(lhs - rhs).max() < 1e-11 * max(1.0, np.abs(rhs).max())


@pytest.mark.parametrize("mesh,k", [(cartesian_quads(3), 3), (voronoi_lloyd(12, 1), 2), (cartesian_hexes(2), 2)])
def test_local_matrices_symmetric_spd(mesh, k):
    geo = mesh_geometry(mesh, k)
    from oracle.solve import default_eta
    for c in range(mesh.n_cells):
        L = local_hho(mesh, geo, c, default_eta(mesh, k), *_zero(mesh.dim))
        assert np.abs(L.a - L.a.T).max() < 1e-12 * np.abs(L.a).max()
        A_TT = vector_system(L)[0]
        assert np.linalg.eigvalsh(L.a[:L.nT, :L.nT]).min() > 0
        ev = np.linalg.eigvalsh(L.a)
        if np.any(mesh.face_bc[mesh.cell_faces(c)] == 1):
            assert ev.min() > 0                    # Nitsche cell: coercive with the default penalty
        else:                                      # interior cell: kernel = constants only
            assert abs(ev[0]) < 1e-11 * ev[-1] and ev[1] > 1e-8 * ev[-1]
        # the mean pressure row of the cell-velocity coupling vanishes (divergence theorem)
        B_T = vector_system(L)[3]
        assert np.abs(B_T[0]).max() < 1e-12 * np.abs(B_T).max()
        del A_TT
