"""GPU tests of the V-cycle replayed from a captured HIP graph (hho_set_graph).

Inside the graph the coarse GMRES runs a fixed budget of columns with the
convergence test on the device; while the eager coarse solve needs no restart
(budget 64 columns here, the coarse tolerance needs far fewer) the two launch
the same kernels on the same data in the same order, so every FGMRES history
and solution must agree to rounding (1e-13; the replays themselves are
deterministic).  Each test replays the graph over several solves with eager
work in between and checks every replay against the eager solve."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from synth import cartesian_quads, voronoi_lloyd, cartesian_hexes, polynomial_stokes  # noqa: E402
from synth.fields import problem_data  # noqa: E402


def _problem(mesh, k, cond, **kw):
    import paper_2009_13840_amd as H
    P = H.Problem(H.Mesh(mesh), k, cond, rtol=1e-10, coarse_restart=64, **kw)
    P.set_data(*problem_data(polynomial_stokes(mesh.dim, k + 1, 21), None, mesh.dim))
    P.bind("cuda:0")
    P.setup()
    return P


def _same(a, b):
    (xa, ita, ha, ra, oka), (xb, itb, hb, rb, okb) = a, b
    assert oka and okb and ita == itb, (ita, itb)
    dh = np.max(np.abs(ha - hb) / np.abs(ha))
    dx = float(np.linalg.norm((xa - xb).cpu().numpy()) / np.linalg.norm(xa.cpu().numpy()))
    assert dh <= 1e-13 and dx <= 1e-13, (dh, dx)
    return dh, dx


@pytest.mark.parametrize("name,mk,k,cond,opts", [
    ("vor60_k3_v_amg", lambda: voronoi_lloyd(60, 2), 3, "v", dict(coarse_mode="amg")),
    ("vor60_k3_vp_fp32", lambda: voronoi_lloyd(60, 2), 3, "vp", dict(coarse_mode="amg", precision="fp32")),
    ("quad4_k2_v_dense", lambda: cartesian_quads(4), 2, "v", dict(coarse_mode="dense")),
    ("hex3_k2_vp_gmres", lambda: cartesian_hexes(3), 2, "vp", dict(coarse_mode="gmres")),
    ("vor60_k3_v_direct", lambda: voronoi_lloyd(60, 2), 3, "v", dict(coarse_mode="direct")),
])
def test_graph_replays_equal_eager_solve(name, mk, k, cond, opts):
    import torch
    mesh = mk()
    print(f"[case] graph {name}", flush=True)
    P = _problem(mesh, k, cond, **opts)
    eager = P.solve()
    P.set_graph(True)
    for rep in range(3):
        got = P.solve()
        dh, dx = _same(eager, got)
        print(f"[graph] {name} replay solve {rep}: its {got[1]}, history diff {dh:.1e}, solution diff {dx:.1e}")
        # eager work of the program between replays
        P.set_graph(False)
        again = P.solve()
        _same(eager, again)
        P.set_graph(True)
        torch.cuda.synchronize()


def test_graph_batch_members_equal_eager():
    import paper_2009_13840_amd as H
    meshes = [cartesian_quads(4), voronoi_lloyd(30, 3), cartesian_quads(6)]
    k = 2
    print("[case] graph batch", flush=True)
    probs = []
    for i, m in enumerate(meshes):
        Q = H.Problem(H.Mesh(m), k, "v", rtol=1e-10, coarse_mode="amg", coarse_restart=64)
        Q.set_data(*problem_data(polynomial_stokes(2, k + 1, 30 + i), None, 2))
        probs.append(Q)
    B = H.Batch(probs)
    B.problem.bind("cuda:0")
    B.problem.setup()
    eager = B.solve(hist_cap=300)
    B.problem.set_graph(True)
    for rep in range(2):
        got = B.solve(hist_cap=300)
        for i in range(len(meshes)):
            fa, pa, ita, ha, ra, sa = eager[i]
            fb, pb, itb, hb, rb, sb = got[i]
            assert sa == 0 and sb == 0 and ita == itb
            assert np.max(np.abs(np.asarray(ha) - np.asarray(hb)) / np.asarray(ha)) <= 1e-13
            assert np.linalg.norm(fa - fb) <= 1e-13 * np.linalg.norm(fa)
        print(f"[graph batch] replay solve {rep}: member its {[g[2] for g in got]}")
