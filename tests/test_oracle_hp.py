"""Pins of the oracle's HHO-hp scheme (Section 2.3.2, Scheme 2: cell velocity one
degree above the face velocity, hybrid pressure), CPU only:

* polynomial solutions (divergence-free u in P^{k+1}, p in P^k) are reproduced
  to rounding by the cell velocity, the cell pressure and the face pressure,
  with Dirichlet and mixed boundaries, in 2D and 3D;
* the global matrix is symmetric and, with a pure Dirichlet boundary, the
  constant pressure (p_T = p_F = 1) is in its kernel;
* the cell velocity is pointwise divergence free for a non-polynomial forcing
  (the property the paper states for this scheme);
* the v&p-cond solve (skeletal unknowns only) with recovery of the cell
  unknowns equals the uncondensed solve;
* convergence under refinement: cell velocity L2 error ~ h^{k+2}, its broken
  gradient ~ h^{k+1}, cell pressure ~ h^{k+1} (at least)."""
import numpy as np
import pytest

from synth import cartesian_quads, voronoi_lloyd, cartesian_hexes, polynomial_stokes, stokes_sincos_2d, trig_series
from synth.fields import problem_data
import oracle.hho_hp as HP


def _neumann_right(mesh):
    return mesh.with_bc(lambda x: 2 if x[0] > 1 - 1e-12 else 1)


def _errors(P, x, man):
    eu = nu = ep = npr = eg = ng = 0.0
    for c in range(P.mesh.n_cells):
        u, gu, div, p, w = HP.cell_fields(P, x, c)
        q = P.locs[c].qpts
        ue, pe, ge = man.u(q), man.p(q), man.grad_u(q)
        eu += w @ ((u - ue) ** 2).sum(1)
        nu += w @ (ue ** 2).sum(1)
        eg += w @ ((gu - ge) ** 2).sum((1, 2))
        ng += w @ (ge ** 2).sum((1, 2))
        ep += w @ (p - pe) ** 2
        npr += w @ pe ** 2
    efp = nfp = 0.0
    for f in range(P.mesh.n_faces):
        pf, xf, wf = HP.face_pressure(P, x, f)
        pe = man.p(xf)
        efp += wf @ (pf - pe) ** 2
        nfp += wf @ pe ** 2
    return {k: np.sqrt(v) for k, v in dict(u=eu, u_norm=nu, grad=eg, grad_norm=ng, p=ep, p_norm=npr,
                                           pF=efp, pF_norm=nfp).items()}


CASES = [
    (cartesian_quads(3), 0), (cartesian_quads(3), 1), (cartesian_quads(3), 3), (voronoi_lloyd(12, 1), 2),
    (_neumann_right(cartesian_quads(3)), 1), (_neumann_right(voronoi_lloyd(10, 4)), 2), (cartesian_hexes(2), 1),
]


@pytest.mark.parametrize("mesh,k", CASES)
def test_hp_polynomial_solution_reproduced(mesh, k):
    man = polynomial_stokes(mesh.dim, k, seed=7)
    P = HP.build_hp(mesh, k, problem_data(man, None, mesh.dim))
    x = HP.normalise_pressure(P, HP.solve_uncondensed(P))
    e = _errors(P, x, man)
    assert e["u"] <= 1e-11 * e["u_norm"]
    assert e["grad"] <= 1e-10 * e["grad_norm"]
    assert e["p"] <= 1e-10 * max(1.0, e["p_norm"])
    assert e["pF"] <= 1e-9 * max(1.0, e["pF_norm"])


@pytest.mark.parametrize("mesh,k", [(voronoi_lloyd(12, 1), 1), (cartesian_hexes(2), 1),
                                    (_neumann_right(cartesian_quads(3)), 2)])
def test_hp_matrix_symmetric_with_constant_pressure_kernel(mesh, k):
    P = HP.build_hp(mesh, k, problem_data(None, trig_series(mesh.dim, 3), mesh.dim))
    A, _ = HP.assemble_full(P)
    scale = abs(A).max()
    assert abs(A - A.T).max() <= 1e-13 * scale
    if P.z is None:                      # a Neumann side: the constant pressure is not in the kernel
        z = np.zeros(P.N)
        for f in range(mesh.n_faces):
            z[P.NU + f * P.locs[0].nF] = np.sqrt(P.geo.faces[f].area)
        for c in range(mesh.n_cells):
            z[P.NU + P.NP + P.NV + c * P.locs[0].nT] = np.sqrt(P.geo.cells[c].volume)
        assert abs(A @ z).max() > 1e-3 * scale * np.abs(z).max()
    else:
        assert abs(A @ P.z).max() <= 1e-13 * scale * np.abs(P.z).max()


@pytest.mark.parametrize("mesh,k", [(voronoi_lloyd(30, 3), 1), (cartesian_quads(4), 2), (cartesian_hexes(2), 1),
                                    (_neumann_right(voronoi_lloyd(20, 5)), 2)])
def test_hp_velocity_is_pointwise_divergence_free(mesh, k):
    P = HP.build_hp(mesh, k, problem_data(None, trig_series(mesh.dim, 11), mesh.dim))
    x = HP.solve_condensed(P)
    dv = gn = 0.0
    for c in range(mesh.n_cells):
        _, gu, div, _, w = HP.cell_fields(P, x, c)
        dv += w @ div ** 2
        gn += w @ (gu ** 2).sum((1, 2))
    assert gn > 0 and np.sqrt(dv / gn) <= 1e-12


@pytest.mark.parametrize("mesh,k", [(voronoi_lloyd(12, 2), 2), (cartesian_hexes(2), 1),
                                    (_neumann_right(cartesian_quads(3)), 1)])
def test_hp_condensed_equals_uncondensed(mesh, k):
    P = HP.build_hp(mesh, k, problem_data(None, trig_series(mesh.dim, 5), mesh.dim))
    xu = HP.normalise_pressure(P, HP.solve_uncondensed(P))
    xc = HP.normalise_pressure(P, HP.solve_condensed(P))
    assert np.abs(xc - xu).max() <= 1e-9 * np.abs(xu).max()


@pytest.mark.parametrize("k", [0, 1])
def test_hp_convergence_rates(k):
    man = stokes_sincos_2d()
    errs = []
    for n in (4, 8, 16):
        P = HP.build_hp(cartesian_quads(n), k, problem_data(man, None, 2))
        errs.append(_errors(P, HP.normalise_pressure(P, HP.solve_condensed(P)), man))
    for key, rate in (("u", k + 2), ("grad", k + 1), ("p", k + 1)):
        r = np.log2(errs[-2][key] / errs[-1][key])
        assert r > rate - 0.15, (key, r)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_hp_viscous_form_from_its_definition_on_the_unit_square(k):
    """The local viscous form a(v, v) (consistency plus face-residual
    stabilisation; all faces Neumann, so no Nitsche terms) against its definition
    evaluated independently: monomials, tensor Gauss-Legendre rules from NumPy,
    the reconstruction solved in the monomial basis and the face residual
    pi_F^k(v_F - p v) - (v_T - p v)|_F formed on each side's parameter.  A face
    residual that projected its cell part onto P^k(F) (the stabilisation of
    equal-order HDG) would differ."""
    mesh = cartesian_quads(1).with_bc(lambda x: 2)
    zero = problem_data(None, trig_series(2, 1), 2)
    P = HP.build_hp(mesh, k, zero)
    L, geo = P.locs[0], P.geo
    rng = np.random.default_rng(40 + k)
    g, gw = np.polynomial.legendre.leggauss(k + 6)
    s, sw = 0.5 * (g + 1.0), 0.5 * gw                          # rule on [0, 1]
    X = np.array([[a, b] for a in s for b in s])
    W = np.array([wa * wb for wa in sw for wb in sw])
    E = [(a, b) for a in range(k + 2) for b in range(k + 2 - a)]
    mono = lambda Y: np.stack([Y[:, 0] ** a * Y[:, 1] ** b for a, b in E], 1)
    dmono = lambda Y: np.stack([np.stack([a * Y[:, 0] ** max(a - 1, 0) * Y[:, 1] ** b,
                                          b * Y[:, 0] ** a * Y[:, 1] ** max(b - 1, 0)], 1) for a, b in E], 1)
    cT = rng.standard_normal(len(E))                           # v_T in P^{k+1}
    sides = []
    for f in geo.cells[0].faces:
        A, B = geo.faces[f].verts
        Y = A[None, :] + s[:, None] * (B - A)[None, :]
        mid = 0.5 * (A + B)
        n = (mid - 0.5) / np.linalg.norm(mid - 0.5)
        cF = rng.standard_normal(k + 1)                        # v_F in P^k(F), in the side parameter
        sides.append((f, Y, n, np.stack([s ** j for j in range(k + 1)], 1) @ cF))
    # reconstruction p v = sum d_m x^m: stiffness and right-hand side in monomials
    G = dmono(X)
    K = np.einsum("q,qid,qjd->ij", W, G, G)
    rhs = np.einsum("q,qid,qd->i", W, G, np.einsum("qjd,j->qd", G, cT))
    for f, Y, n, vF in sides:
        rhs += np.einsum("q,qi->i", sw * (vF - mono(Y) @ cT), dmono(Y) @ n)
    dcoef = np.zeros(len(E))
    dcoef[1:] = np.linalg.solve(K[1:, 1:], rhs[1:])
    dcoef[0] = W @ (mono(X) @ (cT - dcoef))                    # same mean as v_T (E[0] is the constant)
    a_def = W @ (np.einsum("qid,i->qd", G, dcoef) ** 2).sum(1)
    Vk = np.stack([s ** j for j in range(k + 1)], 1)
    Gf = Vk.T @ (sw[:, None] * Vk)
    for f, Y, n, vF in sides:
        pv, vT = mono(Y) @ dcoef, mono(Y) @ cT
        proj = Vk @ np.linalg.solve(Gf, Vk.T @ (sw * (vF - pv)))
        r = proj - (vT - pv)
        a_def += sw @ r ** 2                                   # |F| = h_F = 1
    # the same v in the oracle's local unknowns (orthonormal bases: L2 moments)
    vl = np.zeros(L.nloc)
    vl[:L.N1] = np.einsum("q,qi,q->i", W, L.basis.values(X), mono(X) @ cT)
    for i, (f, Y, n, vF) in enumerate(sides):
        vl[L.N1 + i * L.nF:L.N1 + (i + 1) * L.nF] = np.einsum("q,qj,q->j", sw, geo.face_basis[f].values(Y), vF)
    assert abs(vl @ L.a @ vl - a_def) <= 1e-12 * a_def


@pytest.mark.parametrize("mesh,k", [(voronoi_lloyd(20, 3), 2), (cartesian_hexes(2), 1),
                                    (_neumann_right(cartesian_quads(3)), 2)])
def test_hp_levels_are_galerkin_products_and_keep_the_kernel(mesh, k):
    """Level l + 1 of the skeletal hierarchy is P^T S_l P with P injecting the
    leading P^{k_{l+1}}(F) modes of every face's d velocity components and its
    pressure (built here by explicit loops); with a pure Dirichlet boundary each
    level's constant face pressure is in its kernel."""
    import scipy.sparse as sp
    P = HP.build_hp(mesh, k, problem_data(None, trig_series(mesh.dim, 3), mesh.dim))
    Q, _ = HP.multilevel_problem(P)
    d, nf = mesh.dim, mesh.n_faces
    from math import comb
    for l in range(len(Q.S) - 1):
        nFf, nFc = comb(Q.degrees[l] + d - 1, d - 1), comb(Q.degrees[l + 1] + d - 1, d - 1)
        r = [(f * (d + 1) + cc) * nFf + j for f in range(nf) for cc in range(d + 1) for j in range(nFc)]
        c = [(f * (d + 1) + cc) * nFc + j for f in range(nf) for cc in range(d + 1) for j in range(nFc)]
        Pm = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(nf * (d + 1) * nFf, nf * (d + 1) * nFc))
        G = (Pm.T @ Q.S[l] @ Pm).toarray()
        assert np.abs(G - Q.S[l + 1].toarray()).max() <= 1e-14 * np.abs(G).max()
    for S, z in zip(Q.S, Q.z):
        if P.z is None:
            assert z is None
        else:
            assert np.abs(S @ z).max() <= 1e-11 * abs(S).max() * np.abs(z).max()


@pytest.mark.parametrize("mesh,k", [(voronoi_lloyd(40, 3), 1), (voronoi_lloyd(30, 2), 2), (cartesian_hexes(3), 1),
                                    (_neumann_right(voronoi_lloyd(40, 3)), 2)])
def test_hp_fgmres_vcycle_reaches_the_direct_solution(mesh, k):
    """The p-multilevel solver on the HHO-hp skeleton (levels k..0, cell-patch
    Schwarz smoothing over the faces of each cell, exact coarsest solve): FGMRES
    converges, and the cell unknowns recovered from its skeletal solution are the
    uncondensed solution."""
    import oracle.solve as OS
    P = HP.build_hp(mesh, k, problem_data(None, trig_series(mesh.dim, 7), mesh.dim))
    Q, perm = HP.multilevel_problem(P)
    x, its, hist, conv = OS.solve_fgmres(Q, rtol=1e-11)
    assert conv and its <= 60
    full = HP.normalise_pressure(P, HP.recover_from_skeleton(P, x, perm))
    xu = HP.normalise_pressure(P, HP.solve_uncondensed(P))
    assert np.abs(full - xu).max() <= 1e-6 * np.abs(xu).max()


def test_hp_one_level_vcycle_is_the_skeletal_direct_solve():
    """With a single level the V-cycle is the bordered direct solve of the
    skeleton: FGMRES converges in one iteration."""
    import oracle.solve as OS
    mesh = voronoi_lloyd(16, 9)
    P = HP.build_hp(mesh, 1, problem_data(None, trig_series(2, 4), 2))
    Q, perm = HP.multilevel_problem(P, degrees=[1])
    x, its, hist, conv = OS.solve_fgmres(Q, rtol=1e-10)
    assert conv and its == 1


@pytest.mark.parametrize("mesh,k", [(cartesian_quads(4), 1), (cartesian_quads(3), 2), (voronoi_lloyd(20, 3), 1)])
def test_hp_skeleton_size_and_pattern_match_the_table_formulas(mesh, k):
    """The v&p-cond skeleton of Scheme 2 has the DOF and MNZ counts of the
    paper's tables for HHO-hp (Table tab:DOFsMNZsFormula; the formula is pinned
    against the printed table values by the golden file of the DOF/MNZ test):
    (d + 1) dim P^k(F) unknowns per face, one dense block per pair of faces of a
    common cell."""
    from oracle.system import counts
    P = HP.build_hp(mesh, k, problem_data(None, trig_series(2, 1), 2))
    Sg, _, _ = HP.condense_vp(P)
    c = counts(mesh, k)
    assert Sg.shape[0] == c["dof_hp"] and Sg.nnz == c["mnz_hp"]


@pytest.mark.parametrize("mesh,k", [(voronoi_lloyd(40, 3), 1), (voronoi_lloyd(30, 2), 2), (cartesian_hexes(3), 1)])
def test_hp_with_the_papers_ilu_smoother(mesh, k):
    """The paper's solver configuration (Section 3.3: smoothing by two
    ILU(0)-preconditioned GMRES iterations) on the HHO-hp skeleton: FGMRES
    reaches the uncondensed solution, in no more iterations than with the
    cell-patch Schwarz smoother on these meshes."""
    import oracle.solve as OS
    P = HP.build_hp(mesh, k, problem_data(None, trig_series(mesh.dim, 7), mesh.dim))
    Q, perm = HP.multilevel_problem(P)
    xu = HP.normalise_pressure(P, HP.solve_uncondensed(P))
    its = {}
    for sm in ("ilu", "schwarz"):
        x, its[sm], _, conv = OS.solve_fgmres(Q, rtol=1e-11, smoother=sm)
        full = HP.normalise_pressure(P, HP.recover_from_skeleton(P, x, perm))
        assert conv and np.abs(full - xu).max() <= 1e-6 * np.abs(xu).max()
    assert its["ilu"] <= its["schwarz"], its
