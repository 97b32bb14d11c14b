"""Pins of the oracle's global solution, condensation, levels and Krylov pieces
(Sections 2.3, 3, 4; Tables tab:dofs2D / tab:mnzs2D).  CPU only."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from synth import (cartesian_quads, voronoi_lloyd, cartesian_hexes, polynomial_stokes,
                   stokes_sincos_2d, trig_series)
from synth.fields import problem_data
from oracle.bases import dim_poly
from oracle.condense import condense_v, condense_vp
from oracle.krylov import gmres_steps, fgmres
from oracle.solve import build, solve_direct, errors, solve_fgmres, recover
from oracle.system import assemble_uncondensed, counts, prolongation, layout

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _neumann_right(mesh):
    return mesh.with_bc(lambda x: 2 if x[0] > 1 - 1e-12 else 1)


P1_CASES = [
    (cartesian_quads(3), 0, "v"), (cartesian_quads(3), 0, "vp"),
    (cartesian_quads(3), 1, "v"), (cartesian_quads(4), 3, "vp"), (cartesian_quads(3), 3, "v"),
    (voronoi_lloyd(12, 1), 2, "v"), (voronoi_lloyd(12, 1), 2, "vp"),
    (_neumann_right(cartesian_quads(3)), 2, "v"), (_neumann_right(voronoi_lloyd(10, 4)), 1, "vp"),
    (cartesian_hexes(2), 1, "v"), (cartesian_hexes(2), 1, "vp"),
]


@pytest.mark.parametrize("mesh,k,cond", P1_CASES)
def test_P1_polynomial_solution_reproduced(mesh, k, cond):
    """A divergence-free u in P^{k+1} with p in P^k is reproduced exactly
    (HHO consistency, Section 2.2) for both condensations, Dirichlet and mixed BCs."""
    man = polynomial_stokes(mesh.dim, k, seed=7)
    P = build(mesh, k, cond, problem_data(man, None, mesh.dim))
    x = solve_direct(P)
    e = errors(P, x, man)
    assert e["u_L2"] < 1e-11 * e["u_norm"]
    assert e["grad_u_L2"] < 1e-10 * e["grad_norm"]
    assert e["p_L2"] < 1e-10 * max(1.0, e["p_norm"])
    assert e["energy"] < 1e-10 * e["grad_norm"]


def test_P2_convergence_rates():
    """Energy/pressure errors ~ h^{k+1}, reconstruction L2 ~ h^{k+2} (Section 5.2.2),
    on the 8x8 k=1 manufactured problem refined twice."""
    man = stokes_sincos_2d()
    errs = []
    for n in (8, 16, 32):
        P = build(cartesian_quads(n), 1, "v", problem_data(man, None, 2))
        errs.append(errors(P, solve_direct(P), man))
    for key, rate in (("energy", 2), ("grad_u_L2", 2), ("u_L2", 3), ("p_L2", 2)):
        r = np.log2(errs[-2][key] / errs[-1][key])
        assert r > rate - 0.15, (key, r)


@pytest.mark.parametrize("mesh,k", [(cartesian_quads(2), 2), (voronoi_lloyd(6, 2), 1), (cartesian_hexes(2), 1)])
def test_P3_condensed_equals_uncondensed(mesh, k):
    """Static condensation does not change the solution (Section 5.4): both
    condensed solves plus cell recovery equal the dense LU of the full system."""
    data = problem_data(None, trig_series(mesh.dim, 11), mesh.dim)
    Pv = build(mesh, k, "v", data)
    A, b = assemble_uncondensed(mesh, Pv.locs)
    d, nT = mesh.dim, dim_poly(mesh.dim, k)
    nf, nc, nF = mesh.n_faces, mesh.n_cells, Pv.lays[0].nF
    # border with the constant-pressure vector of the uncondensed layout
    offP = nf * d * nF + nc * d * nT
    z = np.zeros(A.shape[0])
    for c in range(nc):
        z[offP + c * nT] = np.sqrt(Pv.geo.cells[c].volume)
    Ab = np.block([[A.toarray(), z[:, None]], [z[None, :], np.zeros((1, 1))]])
    xu = np.linalg.solve(Ab, np.concatenate([b, [0.0]]))[:-1]
    for cond in ("v", "vp"):
        P = Pv if cond == "v" else build(mesh, k, "vp", data)
        x = solve_direct(P)
        UT, PT = recover(P, x)
        nFd = nf * d * nF
        scale = np.abs(xu).max()
        assert np.abs(x[:nFd] - xu[:nFd]).max() < 1e-11 * scale
        assert np.abs(UT.ravel() - xu[nFd:offP]).max() < 1e-11 * scale
        assert np.abs(PT.ravel() - xu[offP:]).max() < 1e-10 * scale


def test_P4_condensations_coincide_at_k0():
    """v-cond and v&p-cond give the same global system for k = 0 (remark rem:StatCond)."""
    mesh = voronoi_lloyd(20, 9)
    data = problem_data(None, trig_series(2, 5), 2)
    Pv, Pp = build(mesh, 0, "v", data), build(mesh, 0, "vp", data)
    assert np.abs((Pv.S[0] - Pp.S[0]).toarray()).max() <= 1e-15 * abs(Pv.S[0]).max()
    assert np.abs(Pv.b - Pp.b).max() <= 1e-15 * np.abs(Pv.b).max()


def test_vp_is_schur_of_v_over_nonmean_pressure():
    """Eliminating the non-mean pressure modes from the v-cond local system gives
    the v&p-cond local system (block elimination is associative)."""
    mesh = voronoi_lloyd(8, 3)
    P = build(mesh, 2, "v", problem_data(polynomial_stokes(2, 2, 1), None, 2))
    for L in P.locs:
        Sv, rv = condense_v(L)
        Sp, rp = condense_vp(L)
        nd = Sv.shape[0] - L.nT
        keep = np.r_[0:nd, nd]
        elim = np.arange(nd + 1, Sv.shape[0])
        Sk = Sv[np.ix_(keep, keep)] - Sv[np.ix_(keep, elim)] @ np.linalg.solve(Sv[np.ix_(elim, elim)], Sv[np.ix_(elim, keep)])
        rk = rv[keep] - Sv[np.ix_(keep, elim)] @ np.linalg.solve(Sv[np.ix_(elim, elim)], rv[elim])
        assert np.abs(Sk - Sp).max() < 1e-10 * np.abs(Sp).max()
        assert np.abs(rk - rp).max() < 1e-10 * max(1.0, np.abs(rp).max())


@pytest.mark.parametrize("cond", ["v", "vp"])
def test_P5_P6_P8_levels(cond):
    """Coarse operators by sub-block extraction equal explicit P^T S P (bit-equal),
    recursively and in one step; restriction = transpose of prolongation with unit
    diagonal for the hierarchical orthonormal bases; symmetry; z in ker S_l."""
    mesh = voronoi_lloyd(16, 6)
    P = build(mesh, 3, cond, problem_data(None, trig_series(2, 1), 2))
    Pall = sp.identity(P.S[0].shape[0], format="csr")
    for l in range(len(P.S) - 1):
        Pl = prolongation(P.lays[l], P.lays[l + 1])
        explicit = (Pl.T @ P.S[l] @ Pl).tocsr()
        assert abs(explicit - P.S[l + 1]).max() == 0.0
        Pall = Pall @ Pl
        one_step = (Pall.T @ P.S[0] @ Pall).tocsr()
        assert abs(one_step - P.S[l + 1]).max() == 0.0
        R = Pl.T
        c = np.random.default_rng(l).standard_normal(Pl.shape[1])
        assert np.array_equal(R @ (Pl @ c), c)
    for S, z in zip(P.S, P.z):
        assert abs(S - S.T).max() <= 1e-13 * abs(S).max()
        assert np.abs(S @ z).max() <= 1e-12 * abs(S).max() * np.abs(z).max()


def test_P6_restriction_matrix_from_definition():
    """(int_X psi_i^{l+1} psi_j^{l}) computed by quadrature is the unit-diagonal
    rectangular matrix for the bases used (Section 4.2)."""
    from oracle.hho import mesh_geometry
    from oracle.bases import FaceBasis, CellBasis
    from oracle.geometry import cell_quadrature
    mesh = voronoi_lloyd(10, 2)
    geo3 = mesh_geometry(mesh, 3)
    for f in range(0, mesh.n_faces, 7):
        xf, wf = geo3.face_q[f]
        fine = geo3.face_basis[f].values(xf)
        for kc in (2, 1, 0):
            coarse = FaceBasis(geo3.faces[f], xf, wf, kc).values(xf)
            I = coarse.T @ (wf[:, None] * fine)
            assert np.abs(I - np.eye(*I.shape)).max() < 1e-12
    c = 3
    xq, wq = cell_quadrature(mesh, geo3.cells[c], geo3.faces, 12)
    cg = geo3.cells[c]
    fine = CellBasis(cg.centroid, cg.diam, xq, wq, 3).values(xq)
    for kc in (2, 1, 0):
        coarse = CellBasis(cg.centroid, cg.diam, xq, wq, kc).values(xq)
        I = coarse.T @ (wq[:, None] * fine)
        assert np.abs(I - np.eye(*I.shape)).max() < 1e-12


def test_P7_dof_mnz_counts_match_tables():
    gold = json.load(open(os.path.join(GOLDEN, "dof_mnz_2d.json")))
    for case in gold["cases"]:
        got = counts(cartesian_quads(case["n"]), case["k"])
        for key, val in case.items():
            if key in ("n", "k"):
                continue
            assert float("%.3g" % got[key]) == val, (case["n"], case["k"], key, got[key], val)


def test_P7_counts_match_assembled_structure():
    """The DOF count of the v-cond / v&p systems equals the assembled matrix size."""
    mesh = voronoi_lloyd(30, 1)
    data = problem_data(None, trig_series(2, 1), 2)
    for cond, key in (("v", "dof_v"), ("vp", "dof_vp")):
        P = build(mesh, 2, cond, data)
        assert P.S[0].shape[0] == counts(mesh, 2)[key]


def test_P10_gmres_steps_is_krylov_minimiser():
    """m right-preconditioned GMRES steps return the minimiser of |b - A x| over
    x0 + span{M r0, M A M r0, ...}: compare with a least-squares solve on an
    explicitly generated (non-orthogonal) Krylov basis."""
    rng = np.random.default_rng(0)
    n = 40
    A = rng.standard_normal((n, n)) + n * np.eye(n)
    A = A + A.T
    A[0, 0] = -3.0                                  # indefinite
    Mi = np.diag(1.0 / (1.0 + rng.random(n)))
    b, x0 = rng.standard_normal(n), rng.standard_normal(n)
    r0 = b - A @ x0
    for m in (1, 2, 4):
        x = gmres_steps(lambda v: A @ v, lambda v: Mi @ v, x0, r0, m)
        K = [Mi @ r0]
        for _ in range(m - 1):
            K.append(Mi @ (A @ K[-1]))
        K = np.array(K).T
        y = np.linalg.lstsq(A @ K, r0, rcond=None)[0]
        assert np.abs(x - (x0 + K @ y)).max() < 1e-10 * np.abs(x).max()


def test_P10_fgmres_matches_direct():
    rng = np.random.default_rng(1)
    n = 60
    A = rng.standard_normal((n, n)) + 2 * np.sqrt(n) * np.eye(n)
    b = rng.standard_normal(n)
    x, its, hist, conv = fgmres(lambda v: A @ v, lambda v: v, b, 1e-12, restart=10, maxit=500)
    assert conv and np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-9 * np.abs(x).max()
    assert hist[0] == 1.0 and all(h2 <= h1 * (1 + 1e-12) for h1, h2 in zip(hist, hist[1:10]))


@pytest.mark.parametrize("mesh,k,cond", [(cartesian_quads(8), 1, "v"), (voronoi_lloyd(64, 2), 3, "v"),
                                         (voronoi_lloyd(64, 2), 3, "vp")])
def test_fgmres_vcycle_reaches_direct_solution(mesh, k, cond):
    """FGMRES + one V-cycle per iteration converges to 1e-8 in a mesh-independent
    handful of iterations and agrees with the direct solve."""
    P = build(mesh, k, cond, problem_data(None, trig_series(2, 2), 2))
    xd = solve_direct(P)
    x, its, hist, conv = solve_fgmres(P, rtol=1e-10)
    assert conv and its <= 20
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)
