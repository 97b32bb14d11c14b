"""GPU test of the allocation-free loss-and-gradient entry point
(hho_learned_grad_noalloc) through the C ABI: two calls in a row, the second
with fewer rows, each identical to hho_learned_grad (same kernels, same fixed
summation order, only the work arrays live elsewhere) and within the bfloat16
network's bound of the oracle's network; sizes beyond the fixed array are
refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from synth import cartesian_quads, polynomial_stokes  # noqa: E402
from synth.fields import problem_data  # noqa: E402
from oracle import mlp  # noqa: E402


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_noalloc_gradient_matches_workspace_gradient():
    import torch
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    mesh = cartesian_quads(4)
    k, cond = 2, "v"
    data = problem_data(polynomial_stokes(mesh.dim, k + 1, 3), None, mesh.dim)
    print("[case] quad4_k2_v learned gradient, workspace vs fixed scratch", flush=True)
    P = H.Problem(H.Mesh(mesh), k, cond, learned=1, coarse_mode="dense")
    P.set_data(*data)
    P.bind("cuda:0")
    P.setup()
    O = OS.build(mesh, k, cond, data, eta=None)
    L = mlp.layout(mesh, mesh.dim, O.lays[0].nF, O.lays[0].nP)
    rng = np.random.default_rng(21)
    th = mlp.init_params(L.n_in, L.n_out, rng.random(mlp.HIDDEN * L.n_in), rng.random(L.n_out * mlp.HIDDEN))
    th["b1"] = 0.05 * rng.standard_normal(mlp.HIDDEN)
    th["b2"] = 0.05 * rng.standard_normal(L.n_out)
    th = {kk: v.astype(np.float32).astype(np.float64) for kk, v in th.items()}
    flat = np.concatenate([th["W1"].ravel(), th["b1"], th["W2"].ravel(), th["b2"]]).astype(np.float32)
    P.learned_set_params(flat)
    results = []
    for n in (4096, 1000):   # the second call is smaller: stale rows of the first must not leak in
        X = rng.standard_normal((n, L.n_in)).astype(np.float32)
        T = rng.standard_normal((n, L.n_out)).astype(np.float32)
        Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
        print(f"[call] noalloc gradient over {n} rows", flush=True)
        loss_na, g_na = P.learned_grad(Xd, Td, noalloc=True)
        loss_ws, g_ws = P.learned_grad(Xd, Td)
        assert loss_na == loss_ws
        assert np.array_equal(g_na, g_ws)
        lo, go = mlp.loss_and_grad(th, X.astype(np.float64), T.astype(np.float64))
        assert abs(loss_na - lo) <= 1e-3 * lo          # bfloat16 network: see test_gpu_learned
        gflat = np.concatenate([go[kk].ravel() for kk in ("W1", "b1", "W2", "b2")])
        assert _rel(g_na, gflat) < 1e-2, _rel(g_na, gflat)
        results.append(g_na)
    assert not np.array_equal(results[0], results[1])
    # beyond the fixed array: refused before any device work
    X = torch.zeros((4097, L.n_in), dtype=torch.float32, device="cuda:0")
    T = torch.zeros((4097, L.n_out), dtype=torch.float32, device="cuda:0")
    with pytest.raises(H.HHOError) as e:
        P.learned_grad(X, T, noalloc=True)
    assert e.value.code == -7
