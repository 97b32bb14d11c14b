"""GPU tests of the local HHO operators built on the device (options.local_build
= DEVICE; Sections 2.2.1, 2.2.3, 2.3.1): every cell's record [a | B | rhs_u |
rhs_p] against the oracle's local_hho, on quadrilaterals, Voronoi polygons,
boxes, sheared hexahedra (the tetrahedral quadrature path) and a mesh with
Neumann faces, for k = 0 .. 3 (and k = 5 in 2D); then whole solves against the
host build.

Tolerance: the records are formed in FP64 from the same quadrature rules; the
device's bases (classical Gram-Schmidt twice) and its consistency term
(Y^T Y) differ from the oracle's only in rounding order, amplified by the
conditioning of the scaled monomial Gram matrices and of the reconstruction
stiffness (below 1e4 on these cells): 1e-12 of the largest entry (measured:
at most 1.5e-14)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from synth import cartesian_quads, voronoi_lloyd, cartesian_hexes, polynomial_stokes  # noqa: E402
from synth.fields import problem_data  # noqa: E402


def _sheared_hexes(n):
    m = cartesian_hexes(n)
    m.verts = m.verts.copy()
    m.verts[:, 0] += 0.3 * m.verts[:, 1] + 0.1 * m.verts[:, 2]
    return m


CASES = [
    ("quad3_k1", lambda: cartesian_quads(3), 1),
    ("quad4_k0", lambda: cartesian_quads(4), 0),
    ("vor20_k3", lambda: voronoi_lloyd(20, 3), 3),
    ("vor12_k5", lambda: voronoi_lloyd(12, 4), 5),
    ("hex2_k2", lambda: cartesian_hexes(2), 2),
    ("hex2_k3", lambda: cartesian_hexes(2), 3),
    ("shear2_k1", lambda: _sheared_hexes(2), 1),
    ("quad3_k2_neumann", lambda: cartesian_quads(3).with_bc(lambda x: 2 if x[0] > 1 - 1e-12 else 1), 2),
]


def _device_problem(mesh, k, data, mode="device", **kw):
    import paper_2009_13840_amd as H
    P = H.Problem(H.Mesh(mesh), k, "v", local_build=mode, **kw)
    P.set_data(*data)
    P.bind("cuda:0")
    P.setup()
    return P


@pytest.mark.parametrize("name,mk,k", CASES)
def test_device_local_operators_match_oracle(name, mk, k):
    from oracle.hho import mesh_geometry, local_hho
    from oracle.solve import default_eta
    mesh = mk()
    data = problem_data(polynomial_stokes(mesh.dim, k + 1, 7), None, mesh.dim)
    print(f"[case] device local build {name}", flush=True)
    P = _device_problem(mesh, k, data)
    assert P.timings()["local_ms"] > 0
    geo = mesh_geometry(mesh, k)
    eta = default_eta(mesh, k)
    worst = {"a": 0.0, "B": 0.0, "rhs_u": 0.0, "rhs_p": 0.0}
    for c in range(mesh.n_cells):
        L = local_hho(mesh, geo, c, eta, *data)
        G = P.local_cell(c)
        for key, ref in (("a", L.a), ("B", L.B), ("rhs_u", L.rhs_u), ("rhs_p", L.rhs_p)):
            scale = max(np.abs(ref).max(), 1.0 if key.startswith("rhs") else 0.0)
            if scale == 0:
                assert np.abs(G[key]).max() == 0
                continue
            worst[key] = max(worst[key], np.abs(G[key] - ref).max() / scale)
    print(f"[device local] {name}: max rel err " + ", ".join(f"{k_} {v:.1e}" for k_, v in worst.items()))
    assert max(worst.values()) <= 1e-12, worst


@pytest.mark.parametrize("name,mk,k", [CASES[2], CASES[5], CASES[7]])
def test_device_build_solves_like_host_build(name, mk, k):
    """FGMRES on the device-built operators reaches the host-built problem's
    solution (both solves to 1e-12)."""
    mesh = mk()
    data = problem_data(polynomial_stokes(mesh.dim, k + 1, 8), None, mesh.dim)
    print(f"[case] device vs host build {name}", flush=True)
    Pd = _device_problem(mesh, k, data, rtol=1e-12)
    Ph = _device_problem(mesh, k, data, mode="host", rtol=1e-12)
    xd, itd, _, reld, okd = Pd.solve()
    xh, ith, _, relh, okh = Ph.solve()
    assert okd and okh
    xd, xh = xd.cpu().numpy(), xh.cpu().numpy()
    err = np.linalg.norm(xd - xh) / np.linalg.norm(xh)
    print(f"[device vs host] {name}: its {itd} / {ith}, |x_dev - x_host| / |x_host| {err:.1e}")
    assert abs(itd - ith) <= 1 and err <= 1e-9


def test_device_build_with_caller_moments():
    """hho_set_moments over the device build: the caller's moments replace the
    ones the device forms (here: the device's own, read back, doubled, give
    twice the solution of the linear problem)."""
    mesh = voronoi_lloyd(16, 9)
    k = 2
    data = problem_data(polynomial_stokes(2, k + 1, 9), None, 2)
    print("[case] device build with caller moments", flush=True)
    P = _device_problem(mesh, k, data, rtol=1e-12)
    x1 = P.solve()[0].cpu().numpy()
    ru = np.concatenate([P.local_cell(c)["rhs_u"].ravel() for c in range(mesh.n_cells)])
    rp = np.concatenate([P.local_cell(c)["rhs_p"] for c in range(mesh.n_cells)])
    P.set_moments(2.0 * ru, 2.0 * rp)
    P.setup()
    x2 = P.solve()[0].cpu().numpy()
    assert np.linalg.norm(x2 - 2.0 * x1) <= 1e-9 * np.linalg.norm(x1)
