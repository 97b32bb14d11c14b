"""GPU tests of the paper's smoother (options.smoother = ILU; Section 3.3 and the
solver options of Section 5.2): GMRES(2) right-preconditioned by the zero-fill
ILU of each level operator in the natural ordering, against the oracle
(oracle.ilu.ILU0 on the oracle's level matrices, oracle.solve.hierarchy with
smoother="ilu").

* The preconditioner alone, level by level: z = U^{-1} L^{-1} r.  Both sides
  eliminate row by row in the same order from level operators that agree to
  rounding (1e-12), so z agrees to 1e-12 of its largest entry (the incomplete
  factors amplify the operators' rounding by their conditioning, below 1e2 on
  these levels; measured at most 8e-15).
* FGMRES with the exact coarsest solve: the V-cycle is the same linear map on
  both sides, so the iteration counts are equal and the relative residual
  estimates agree to 1e-8 per entry while above 1e-8.
* With the coarsest level solved by GMRES preconditioned by its ILU (the paper's
  3D coarse solve), FGMRES reaches the direct solution."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from synth import cartesian_quads, voronoi_lloyd, cartesian_hexes, polynomial_stokes  # noqa: E402
from synth.fields import problem_data  # noqa: E402

CASES = [
    ("quad4_k2_v", lambda: cartesian_quads(4), 2, "v"),
    ("vor40_k3_v", lambda: voronoi_lloyd(40, 3), 3, "v"),
    ("vor40_k3_vp", lambda: voronoi_lloyd(40, 3), 3, "vp"),
    ("hex2_k2_vp", lambda: cartesian_hexes(2), 2, "vp"),
    ("hex2_k3_v", lambda: cartesian_hexes(2), 3, "v"),
    ("quad4_k1_v_neumann", lambda: cartesian_quads(4).with_bc(lambda x: 2 if x[0] > 1 - 1e-12 else 1), 1, "v"),
]


@pytest.fixture(scope="module")
def built():
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    cache = {}

    def get(name, mk, k, cond, **opts):
        key = (name, tuple(sorted(opts.items())))
        if key not in cache:
            mesh = mk()
            data = problem_data(polynomial_stokes(mesh.dim, k + 1, 3), None, mesh.dim)
            print(f"[case] ilu {name} {opts}", flush=True)
            P = H.Problem(H.Mesh(mesh), k, cond, smoother="ilu", **opts)
            P.set_data(*data)
            P.bind("cuda:0")
            P.setup()
            O = OS.build(mesh, k, cond, data, eta=None)
            cache[key] = (mesh, P, O)
        return cache[key]
    return get


@pytest.mark.parametrize("name,mk,k,cond", CASES)
def test_ilu_preconditioner_matches_oracle(built, name, mk, k, cond):
    import torch
    from oracle.ilu import ILU0
    mesh, P, O = built(name, mk, k, cond, coarse_mode="dense", rtol=1e-10)
    rng = np.random.default_rng(51)
    for l in range(len(O.S) - 1):           # the smoothed levels
        r = rng.standard_normal(O.S[l].shape[0])
        want = ILU0(O.S[l])(r)
        got = P.precond_apply(l, torch.from_numpy(r).cuda()).cpu().numpy()
        err = np.abs(got - want).max() / np.abs(want).max()
        print(f"[ilu] {name} level {l}: max |z - z_oracle| / max |z_oracle| {err:.1e}")
        assert err <= 1e-12, (l, err)


@pytest.mark.parametrize("name,mk,k,cond", CASES)
def test_ilu_smoothed_fgmres_history_matches_oracle(built, name, mk, k, cond):
    import oracle.solve as OS
    mesh, P, O = built(name, mk, k, cond, coarse_mode="dense", rtol=1e-10)
    x, its, hist, rel, ok = P.solve()
    assert ok
    xo, its_o, hist_o, conv = OS.solve_fgmres(O, rtol=1e-10, coarse="direct", smoother="ilu")
    ho = np.asarray(hist_o)
    print(f"[ilu history] {name}: its {its} (oracle {its_o})")
    assert its == its_o and len(hist) == len(ho)
    sel = ho > 1e-8
    dev = np.abs(hist[sel] - ho[sel]) / ho[sel]
    print(f"[ilu history] {name}: max per-entry deviation {dev.max():.2e}")
    assert dev.max() <= 1e-8, dev.max()


@pytest.mark.parametrize("name,mk,k,cond", [CASES[1], CASES[3]])
def test_ilu_gmres_coarse_reaches_direct_solution(built, name, mk, k, cond):
    import oracle.solve as OS
    mesh, P, O = built(name, mk, k, cond, coarse_mode="gmres", rtol=1e-12)
    x, its, hist, rel, ok = P.solve()
    assert ok and rel <= 1e-12
    xd = OS.normalise_pressure(O, OS.solve_direct(O))
    nf = O.lays[0].off
    err = np.linalg.norm(x.cpu().numpy()[:nf] - xd[:nf]) / np.linalg.norm(xd[:nf])
    print(f"[ilu coarse gmres] {name}: its {its}, face error vs direct {err:.1e}")
    assert err <= 1e-9


def test_ilu_smoother_in_a_batch_and_in_a_graph():
    """The ILU smoother inside a batch (the union's factors are the members'
    own: the operator is block diagonal and the natural ordering keeps each
    member's unknowns together) gives every member the oracle's direct solution,
    and the V-cycle replayed from a graph gives the eager iterates exactly."""
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    meshes = [cartesian_quads(4), voronoi_lloyd(30, 3)]
    k = 2
    fields = [problem_data(polynomial_stokes(2, k + 1, 60 + i), None, 2) for i in range(2)]
    print("[case] ilu batch", flush=True)
    probs = []
    for m, f in zip(meshes, fields):
        Q = H.Problem(H.Mesh(m), k, "v", smoother="ilu", coarse_mode="amg", rtol=1e-12, coarse_restart=64)
        Q.set_data(*f)
        probs.append(Q)
    B = H.Batch(probs)
    B.problem.bind("cuda:0")
    B.problem.setup()
    eager = B.solve(hist_cap=300)
    for i, (m, f) in enumerate(zip(meshes, fields)):
        face, pres, its, hist, rel, status = eager[i]
        O = OS.build(m, k, "v", f, eta=None)
        xd = OS.normalise_pressure(O, OS.solve_direct(O))
        ef = np.linalg.norm(face - xd[:face.size]) / np.linalg.norm(xd[:face.size])
        print(f"[ilu batch] member {i}: its {its}, face error vs direct {ef:.1e}")
        assert status == 0 and ef <= 1e-9
    B.problem.set_graph(True)
    got = B.solve(hist_cap=300)
    for i in range(len(meshes)):
        assert got[i][2] == eager[i][2]
        assert np.array_equal(np.asarray(got[i][3]), np.asarray(eager[i][3]))
