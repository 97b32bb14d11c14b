"""Batched solves through the C ABI: several independent problems as one
disjoint-union problem with one FGMRES process per member.  Every member's
solution must equal the oracle's direct solve of that member alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from synth import cartesian_quads, voronoi_lloyd, cartesian_hexes, polynomial_stokes, trig_series  # noqa: E402
from synth.fields import problem_data  # noqa: E402
from synth.batch import shifted, region_fields  # noqa: E402


@pytest.mark.parametrize("dim,k,cond", [(2, 2, "v"), (2, 1, "vp"), (3, 1, "v")])
def test_batched_members_match_oracle(dim, k, cond):
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    if dim == 2:
        members = [cartesian_quads(4), voronoi_lloyd(30, 3), cartesian_quads(6), voronoi_lloyd(18, 8)]
    else:
        members = [cartesian_hexes(2), cartesian_hexes(3)]
    # polynomial data (exact quadrature on both sides), a different solution per member
    fields = [problem_data(polynomial_stokes(dim, k + 1, 40 + i), None, dim) for i in range(len(members))]
    width = 2.0
    U, fo, co = H.Mesh.union([shifted(m, width * i) for i, m in enumerate(members)])
    print(f"[case] batch dim={dim} k={k} {cond}: {len(members)} members, {U.n_cells} cells", flush=True)
    P = H.Problem(U, k, cond, rtol=1e-12)
    P.set_segments(fo, co)
    P.set_data(*region_fields(fields, dim, width))
    P.bind("cuda:0")
    P.setup()
    x, its, hist, rel, ok = P.solve()
    assert ok and rel <= 1e-12
    m_its, m_rel = P.batch_results()
    assert np.all(m_rel <= 1e-12) and np.all(m_its >= 1) and m_its.max() == its
    x = x.cpu().numpy()
    # members solved to 1e-12; the shifted geometry (member i at x + 2i) perturbs
    # the local operators at rounding level, so solutions agree to ~1e-10
    lay_dp = None
    n0 = P.level_size(0)
    nface_total = int(fo[-1])
    # every member takes its own default penalty, as it would alone
    for i, mesh in enumerate(members):
        O = OS.build(mesh, k, cond, fields[i], eta=None)
        xd = OS.normalise_pressure(O, OS.solve_direct(O))
        nF, nP = O.lays[0].nF, O.lays[0].nP
        dp = dim * nF
        lay_dp = dp
        xf = x[fo[i] * dp:fo[i + 1] * dp]
        xc = x[nface_total * dp + co[i] * nP:nface_total * dp + co[i + 1] * nP]
        xm = np.concatenate([xf, xc])
        assert xm.shape == xd.shape
        err = np.linalg.norm(xm - xd) / np.linalg.norm(xd)
        print(f"[member] {i}: its {m_its[i]} rel {m_rel[i]:.2e} |x - x_direct|/|x| {err:.2e}")
        assert err <= 1e-8, (i, err)
    assert n0 == nface_total * lay_dp + int(co[-1]) * nP


def test_batched_restart_after_a_member_converged():
    """Members of very different difficulty with a short restart: the easy member
    converges while the hard one still restarts.  The converged member's basis
    vectors must stay zero (they feed the union-wide V-cycle); every member
    converges and no breakdown is reported."""
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    members = [cartesian_quads(2), voronoi_lloyd(60, 11), cartesian_quads(3), voronoi_lloyd(45, 12)]
    fields = [problem_data(polynomial_stokes(2, 3, 70 + i), None, 2) for i in range(len(members))]
    width = 2.0
    U, fo, co = H.Mesh.union([shifted(m, width * i) for i, m in enumerate(members)])
    print(f"[case] batch restart=4, {len(members)} members, {U.n_cells} cells", flush=True)
    P = H.Problem(U, 2, "v", rtol=1e-10, restart=4, coarse_mode="gmres")
    P.set_segments(fo, co)
    P.set_data(*region_fields(fields, 2, width))
    P.bind("cuda:0")
    P.setup()
    x, its, hist, rel, ok = P.solve()
    m_its, m_rel = P.batch_results()
    print(f"[members] its {m_its.tolist()} rel {m_rel.tolist()}")
    assert ok and np.all(m_rel <= 1e-10), (m_its, m_rel)
    assert m_its.min() < m_its.max()      # the members really converge at different times
    assert m_its.max() > 4                # and the slowest restarts at least once
    x = x.cpu().numpy()
    nface_total = int(fo[-1])
    for i, mesh in enumerate(members):
        O = OS.build(mesh, 2, "v", fields[i])
        xd = OS.normalise_pressure(O, OS.solve_direct(O))
        dp, nP = 2 * O.lays[0].nF, O.lays[0].nP
        xm = np.concatenate([x[fo[i] * dp:fo[i + 1] * dp],
                             x[nface_total * dp + co[i] * nP:nface_total * dp + co[i + 1] * nP]])
        err = np.linalg.norm(xm - xd) / np.linalg.norm(xd)
        assert err <= 1e-7, (i, err)



def _batch_run(meshes, fields, k, cond, **opts):
    import paper_2009_13840_amd as H
    probs = []
    for m, f in zip(meshes, fields):
        Q = H.Problem(H.Mesh(m), k, cond, **opts)
        Q.set_data(*f)
        probs.append(Q)
    B = H.Batch(probs)
    B.problem.bind("cuda:0")
    B.problem.setup()
    return B.solve(hist_cap=400)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_member_does_not_depend_on_its_companions(precision):
    """Inside the V-cycle every member takes its own minimal-residual smoothing
    coefficients and runs its own coarse GMRES (Section 3.3's V-cycle per
    member), as the outer FGMRES already does: with a preconditioner that has no
    union-wide quantity (Schwarz-preconditioned coarse GMRES), a member's
    iteration count, residual history and solution are the same whichever
    problems share its batch and at whatever position; alone (the
    single-problem kernels sum in another order) it takes the same iterations
    and its history agrees while above the tolerance."""
    import paper_2009_13840_amd as H
    k, cond = 2, "v"
    A = voronoi_lloyd(30, 3)
    others = [cartesian_quads(6), voronoi_lloyd(45, 5), cartesian_quads(3)]
    fA = problem_data(polynomial_stokes(2, k + 1, 81), None, 2)
    fo = [problem_data(polynomial_stokes(2, k + 1, 82 + i), None, 2) for i in range(3)]
    opts = dict(rtol=1e-10, coarse_mode="gmres", precision=precision)
    print(f"[case] member independence, precision={precision}", flush=True)
    r1 = _batch_run([A, others[0]], [fA, fo[0]], k, cond, **opts)[0]
    r2 = _batch_run([others[1], A, others[2]], [fo[1], fA, fo[2]], k, cond, **opts)[1]
    face1, pres1, its1, h1, rel1, st1 = r1
    face2, pres2, its2, h2, rel2, st2 = r2
    dh = np.max(np.abs(np.asarray(h1) - np.asarray(h2)) / np.asarray(h1))
    print(f"[member A] its {its1} / {its2}, history max rel diff {dh:.2e}")
    assert st1 == 0 and st2 == 0
    assert its1 == its2 and dh <= 1e-12
    assert np.linalg.norm(face1 - face2) <= 1e-13 * np.linalg.norm(face1)
    # alone
    P = H.Problem(H.Mesh(A), k, cond, **opts)
    P.set_data(*fA)
    P.bind("cuda:0")
    P.setup()
    x, its, hist, rel, ok = P.solve(hist_cap=400)
    hist = np.asarray(hist)
    print(f"[member A alone] its {its}")
    assert ok and its == its1
    above = hist > 1e-8
    assert np.all(np.abs(hist[above] - np.asarray(h1)[above]) <= 1e-6 * hist[above])
    nf = face1.size
    assert np.linalg.norm(x.cpu().numpy()[:nf] - face1) <= 1e-8 * np.linalg.norm(face1)
