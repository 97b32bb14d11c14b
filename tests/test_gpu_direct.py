"""GPU tests of the sparse direct coarse solver (options.coarse_mode = "direct";
the paper's 2D coarse solver is a direct factorisation, Section 5.2).

* The coarse solve alone (hho_coarse_solve_apply) against the oracle's bordered
  direct solve of its coarsest operator (oracle.multilevel.Hierarchy with
  coarse = "direct": the LU of [S z; z^T 0]), on meshes whose elimination trees
  have fronts eliminated in LDS and fronts eliminated by panels, v- and
  v&p-cond, with and without the pressure null space: both are exact solves
  and differ by rounding amplified by the coarse operator's conditioning, so
  1e-10 of the largest entry.
* At the full size of the benchmark's 2D workload (16384 Voronoi cells, k = 3,
  v-cond): properties that hold at any size — for b = S y (y random) the
  solution x satisfies S x = b to 1e-10 relative, and x is orthogonal to the
  constant-pressure null vector.
* The whole solver with the direct coarse solve, in a batch of problems with a
  Neumann boundary (no null space) or of pure-Dirichlet problems (a pinned
  pressure and a projection per member), reaches every member's direct
  solution."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from synth import cartesian_quads, voronoi_lloyd, cartesian_hexes, polynomial_stokes  # noqa: E402
from synth.fields import problem_data  # noqa: E402


def _neumann(m):
    return m.with_bc(lambda x: 2 if x[0] > 1 - 1e-12 else 1)


CASES = [
    ("vor600_k1_v", lambda: voronoi_lloyd(600, 4), 1, "v"),
    ("vor600_k1_vp", lambda: voronoi_lloyd(600, 4), 1, "vp"),
    ("quad16_k1_v_neumann", lambda: _neumann(cartesian_quads(16)), 1, "v"),
    ("hex6_k1_vp", lambda: cartesian_hexes(6), 1, "vp"),
    ("hex5_k1_v", lambda: cartesian_hexes(5), 1, "v"),
    ("quad3_k2_v", lambda: cartesian_quads(3), 2, "v"),      # one front, no panel
    # one cell with a Neumann side: one front, nothing pinned (with an all-Dirichlet
    # boundary the one cell's smoother patch is singular, rejected at setup)
    ("quad1_k1_v_neumann", lambda: _neumann(cartesian_quads(1)), 1, "v"),
]


@pytest.mark.parametrize("name,mk,k,cond", CASES)
def test_direct_coarse_solve_matches_oracle(name, mk, k, cond):
    import torch
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    mesh = mk()
    data = problem_data(polynomial_stokes(mesh.dim, k + 1, 4), None, mesh.dim)
    print(f"[case] direct coarse solve {name}", flush=True)
    P = H.Problem(H.Mesh(mesh), k, cond, coarse_mode="direct")
    P.set_data(*data)
    P.bind("cuda:0", fill=0xFF)        # NaN bytes: a read of unwritten workspace shows up
    P.setup()
    sizes = P.direct_info("sizes")
    O = OS.build(mesh, k, cond, data, eta=None)
    Hh = OS.hierarchy(O, coarse="direct")
    rng = np.random.default_rng(8)
    L = len(O.S) - 1
    for rep in range(2):
        b = rng.standard_normal(O.S[L].shape[0])
        want = Hh.coarse_solve(b)
        got = P.coarse_solve_apply(torch.from_numpy(b).cuda()).cpu().numpy()
        err = np.abs(got - want).max() / np.abs(want).max()
        print(f"[direct] {name}: {sizes[0]} fronts, {sizes[1]} heights, largest front {sizes[4]}, "
              f"max |x - x_oracle| / max |x_oracle| {err:.1e}")
        assert np.isfinite(got).all() and err <= 1e-10, err


def test_direct_coarse_solve_at_full_size():
    import torch
    import paper_2009_13840_amd as H
    mesh = voronoi_lloyd(16384, 2)
    k = 3
    print("[case] direct coarse solve at full size (16384 Voronoi cells)", flush=True)
    P = H.Problem(H.Mesh(mesh), k, "v", coarse_mode="direct")
    P.set_data(*problem_data(polynomial_stokes(2, k + 1, 5), None, 2))
    P.bind("cuda:0")
    P.setup()
    Lc = P.nlev - 1
    n = P.level_size(Lc)
    y = torch.from_numpy(np.random.default_rng(9).standard_normal(n)).cuda()
    b = P.level_apply(Lc, y)
    x = P.coarse_solve_apply(b)
    r = P.level_apply(Lc, x) - b
    rel = float(torch.linalg.norm(r) / torch.linalg.norm(b))
    # null vector: |T|^{1/2} on each cell's pressure (convex cells: fan areas)
    V = mesh.verts
    area = np.zeros(mesh.n_cells)
    for c in range(mesh.n_cells):
        fs = mesh.cell_faces(c)
        pts = np.array([V[v] for f in fs for v in mesh.face_vertices(f)])
        ctr = pts.mean(axis=0)
        for f in fs:
            a, bb = V[mesh.face_vertices(f)]
            area[c] += 0.5 * abs((a[0] - ctr[0]) * (bb[1] - ctr[1]) - (a[1] - ctr[1]) * (bb[0] - ctr[0]))
    nface = n - mesh.n_cells
    z = np.zeros(n)
    z[nface:] = np.sqrt(area)
    xc = x.cpu().numpy()
    orth = abs(z @ xc) / (np.linalg.norm(z) * np.linalg.norm(xc))
    print(f"[direct full size] {n} coarse unknowns, {P.direct_info('sizes')[0]} fronts: |S x - b| / |b| {rel:.1e}, "
          f"|z.x| / (|z| |x|) {orth:.1e}")
    assert rel <= 1e-10 and orth <= 1e-12
    xs, its, hist, relf, ok = P.solve()
    print(f"[direct full size] FGMRES: {its} its, rel {relf:.1e}")
    assert ok and relf <= 1e-8


@pytest.mark.parametrize("boundary", ["neumann", "dirichlet"])
def test_direct_coarse_solve_in_a_batch(boundary):
    """Members with a Neumann boundary (no null space) or pure Dirichlet ones
    (one pinned pressure and one projection per member)."""
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    meshes = [cartesian_quads(6), voronoi_lloyd(50, 3), voronoi_lloyd(30, 8)]
    if boundary == "neumann":
        meshes = [_neumann(m) for m in meshes]
    k = 2
    fields = [problem_data(polynomial_stokes(2, k + 1, 70 + i), None, 2) for i in range(len(meshes))]
    print(f"[case] direct coarse solve in a batch ({boundary})", flush=True)
    probs = []
    for m, f in zip(meshes, fields):
        Q = H.Problem(H.Mesh(m), k, "v", coarse_mode="direct", rtol=1e-12)
        Q.set_data(*f)
        probs.append(Q)
    B = H.Batch(probs)
    B.problem.bind("cuda:0")
    B.problem.setup()
    out = B.solve(hist_cap=300)
    for i, (m, f) in enumerate(zip(meshes, fields)):
        face, pres, its, hist, rel, status = out[i]
        O = OS.build(m, k, "v", f, eta=None)
        xd = OS.normalise_pressure(O, OS.solve_direct(O))
        nf = face.size
        ef = np.linalg.norm(face - xd[:nf]) / np.linalg.norm(xd[:nf])
        print(f"[direct batch] member {i}: its {its}, face error vs direct {ef:.1e}")
        assert status == 0 and ef <= 1e-9
