"""GPU tests of the learned fine-level smoother through the C ABI: inference,
training-pair collection, loss gradient and the learned V-cycle against the
CPU oracle (oracle/mlp.py), and what training gains over the plain smoother.

Tolerances: the network runs on bfloat16 inputs, weights and activations with
FP32 sums on the GPU, and on the same bfloat16-rounded values with exact sums in
the oracle (oracle.mlp, quantize=True); the two differ by FP32 rounding, and
where an FP32 pre-activation and its exact value round to different bfloat16
neighbours, by one bfloat16 step of that activation: 1e-2 relative to the
largest entry (the P13 bound), 1e-3 for the loss."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from synth import cartesian_quads, voronoi_lloyd, cartesian_hexes, polynomial_stokes  # noqa: E402
from synth.fields import problem_data  # noqa: E402
from oracle import mlp  # noqa: E402

CASES = [
    ("quad4_k2_v", lambda: cartesian_quads(4), 2, "v"),
    ("vor30_k2_vp", lambda: voronoi_lloyd(30, 4), 2, "vp"),
    ("hex2_k1_v", lambda: cartesian_hexes(2), 1, "v"),
]


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _params(rng, n_in, n_out):
    th = mlp.init_params(n_in, n_out, rng.random(mlp.HIDDEN * n_in), rng.random(n_out * mlp.HIDDEN))
    th["b1"] = 0.05 * rng.standard_normal(mlp.HIDDEN)
    th["b2"] = 0.05 * rng.standard_normal(n_out)
    th = {k: v.astype(np.float32).astype(np.float64) for k, v in th.items()}   # the GPU holds FP32
    flat = np.concatenate([th["W1"].ravel(), th["b1"], th["W2"].ravel(), th["b2"]]).astype(np.float32)
    return th, flat


@pytest.fixture(scope="module")
def built():
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    cache = {}

    def get(name, mk, k, cond):
        if name not in cache:
            mesh = mk()
            data = problem_data(polynomial_stokes(mesh.dim, k + 1, 3), None, mesh.dim)
            print(f"[case] {name} k={k} cond={cond} learned", flush=True)
            P = H.Problem(H.Mesh(mesh), k, cond, learned=1, coarse_mode="dense")
            P.set_data(*data)
            P.bind("cuda:0")
            P.setup()
            O = OS.build(mesh, k, cond, data, eta=None)
            L = mlp.layout(mesh, mesh.dim, O.lays[0].nF, O.lays[0].nP)
            cache[name] = (mesh, P, O, L)
        return cache[name]
    return get


@pytest.mark.parametrize("name,mk,k,cond", CASES)
def test_dims_match_window_definition(built, name, mk, k, cond):
    mesh, P, O, L = built(name, mk, k, cond)
    dm = P.learned_dims()
    assert (dm["n_in"], dm["n_out"], dm["hidden"]) == (L.n_in, L.n_out, mlp.HIDDEN)
    assert dm["n_params"] == mlp.HIDDEN * L.n_in + mlp.HIDDEN + L.n_out * mlp.HIDDEN + L.n_out


@pytest.mark.parametrize("name,mk,k,cond", CASES)
def test_inference_matches_oracle(built, name, mk, k, cond):
    import torch
    mesh, P, O, L = built(name, mk, k, cond)
    rng = np.random.default_rng(11)
    th, flat = _params(rng, L.n_in, L.n_out)
    P.learned_set_params(flat)
    assert np.array_equal(P.learned_get_params(), flat)
    r = rng.standard_normal(O.S[0].shape[0])
    z = P.learned_apply(torch.from_numpy(r).cuda()).cpu().numpy()
    zo = mlp.apply(th, mesh, L, r.astype(np.float32).astype(np.float64))
    print(f"[inference] {name}: faces {_rel(z[:L.nface], zo[:L.nface]):.2e} cells {_rel(z[L.nface:], zo[L.nface:]):.2e}")
    assert _rel(z[:L.nface], zo[:L.nface]) < 1e-2
    assert _rel(z[L.nface:], zo[L.nface:]) < 1e-2
    assert np.abs(z[L.nface:]).max() > 0          # the pressure head corrects the cells


@pytest.mark.parametrize("name,mk,k,cond", CASES)
def test_collect_first_cycle_matches_oracle(built, name, mk, k, cond):
    """With x = 0 the first pair is (window of S x_true, x_true_F / s_F)."""
    import torch
    mesh, P, O, L = built(name, mk, k, cond)
    rng = np.random.default_rng(12)
    xt = rng.standard_normal(O.S[0].shape[0])
    X, T = P.learned_collect(torch.from_numpy(xt).cuda(), 1)
    Xo, so = mlp.windows(mesh, L, O.S[0] @ xt)
    To = mlp.targets(mesh, L, xt, so)
    assert X.shape == Xo.shape and T.shape == To.shape
    assert _rel(X.cpu().numpy(), Xo) < 1e-6, _rel(X.cpu().numpy(), Xo)
    assert _rel(T.cpu().numpy(), To) < 1e-6, _rel(T.cpu().numpy(), To)


@pytest.mark.parametrize("name,mk,k,cond", CASES[:2])
def test_gradient_matches_oracle(built, name, mk, k, cond):
    import torch
    mesh, P, O, L = built(name, mk, k, cond)
    rng = np.random.default_rng(13)
    th, flat = _params(rng, L.n_in, L.n_out)
    P.learned_set_params(flat)
    n = 300
    X = rng.standard_normal((n, L.n_in)).astype(np.float32)
    T = rng.standard_normal((n, L.n_out)).astype(np.float32)
    loss, g = P.learned_grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    lo, go = mlp.loss_and_grad(th, X.astype(np.float64), T.astype(np.float64))
    assert abs(loss - lo) <= 1e-3 * lo
    off = 0
    for key in ("W1", "b1", "W2", "b2"):
        sz = go[key].size
        print(f"[grad] {name} {key}: {_rel(g[off:off + sz], go[key].ravel()):.2e}")
        assert _rel(g[off:off + sz], go[key].ravel()) < 1e-2, (key, _rel(g[off:off + sz], go[key].ravel()))
        off += sz
    assert off == g.size


@pytest.mark.parametrize("name,mk,k,cond", CASES)
def test_learned_vcycle_matches_oracle(built, name, mk, k, cond):
    import torch
    import oracle.solve as OS
    mesh, P, O, L = built(name, mk, k, cond)
    rng = np.random.default_rng(14)
    th, flat = _params(rng, L.n_in, L.n_out)
    P.learned_set_params(flat)
    P.learned_enable(True)
    try:
        H = OS.hierarchy(O, coarse="direct")
        H.learned = lambda r: mlp.apply(th, mesh, L, r)
        b = rng.standard_normal(O.S[0].shape[0])
        if O.z[0] is not None:
            b = OS.project_out(O.z[0])(b)
        x = P.vcycle_apply(torch.from_numpy(b).cuda()).cpu().numpy()
        xo = H.vcycle(0, b)
        if O.z[0] is not None:
            x, xo = OS.project_out(O.z[0])(x), OS.project_out(O.z[0])(xo)
        print(f"[learned vcycle] {name}: {_rel(x, xo):.2e}")
        assert _rel(x, xo) < 1e-2, _rel(x, xo)
    finally:
        P.learned_enable(False)


def _splitmix64(x):
    """SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014)."""
    M = (1 << 64) - 1
    x = (x + 0x9E3779B97F4A7C15) & M
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & M
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & M
    return x ^ (x >> 31)


def _batch_rows(seed, step, B, n):
    """Rows of training step `step` (from 0): SplitMix64(seed xor SplitMix64(step << 32 | i)) mod n."""
    return np.array([_splitmix64(seed ^ _splitmix64((step << 32) | i)) % n for i in range(B)], dtype=np.int64)


@pytest.mark.parametrize("name,mk,k,cond", CASES[:2])
def test_adam_steps_match_oracle(built, name, mk, k, cond):
    """Three training steps: the batch rows follow the documented SplitMix64 draw,
    and the Adam kernel's parameters after each step equal the oracle's Adam
    update (FP64, oracle.mlp.adam_step, bias-corrected moments from zero) applied
    to the gradient the library computes for those rows at its current
    parameters.  Tolerance: FP32 rounding of the update arithmetic, 1e-6 of a
    parameter plus 1e-4 of the learning rate."""
    import torch
    mesh, P, O, L = built(name, mk, k, cond)
    rng = np.random.default_rng(17)
    th, flat = _params(rng, L.n_in, L.n_out)
    P.learned_set_params(flat)
    n, B, lr, seed = 500, 96, 1e-3, 1234567
    X = torch.from_numpy(rng.standard_normal((n, L.n_in)).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.standard_normal((n, L.n_out)).astype(np.float32)).cuda()
    keys = ("W1", "b1", "W2", "b2")
    m = {k_: np.zeros_like(th[k_]) for k_ in keys}
    v = {k_: np.zeros_like(th[k_]) for k_ in keys}
    tho = dict(th)
    for step in range(3):
        rows = torch.from_numpy(_batch_rows(seed, step, B, n)).cuda()
        _, g = P.learned_grad(X[rows].contiguous(), T[rows].contiguous())
        hist = P.learned_train(X, T, steps=1, batch=B, lr=lr, seed=seed)
        assert np.isfinite(hist).all()
        gd, off = {}, 0
        for k_ in keys:
            gd[k_] = g[off:off + th[k_].size].astype(np.float64).reshape(th[k_].shape)
            off += th[k_].size
        tho, m, v = mlp.adam_step(tho, gd, m, v, step + 1, lr)
        want = np.concatenate([tho[k_].ravel() for k_ in keys])
        got = P.learned_get_params().astype(np.float64)
        err = np.abs(got - want) / (1e-6 * np.abs(want) + 1e-4 * lr)
        print(f"[adam] {name} step {step + 1}: worst error / tolerance {err.max():.2f}")
        assert err.max() <= 1.0, err.max()
        # the step really moved the parameters (by about lr where the gradient is not zero)
        moved = np.abs(got - np.concatenate([th[k_].ravel() for k_ in keys]))
        assert moved.max() > 0.5 * lr


def test_training_gain_over_plain_smoother():
    """Trains on V-cycle pairs of a 3D problem and reports the fine-level
    smoothing gain; the learned step can never lose to the plain one (it
    minimises over a superset of directions), and training must lower the loss."""
    import torch
    import paper_2009_13840_amd as H
    from synth import trig_series
    mesh = cartesian_hexes(6)
    k = 2
    data = problem_data(None, trig_series(3, 5), 3)
    P = H.Problem(H.Mesh(mesh), k, "v", learned=1, rtol=1e-10)
    P.set_data(*data)
    P.bind("cuda:0")
    P.setup()
    dm = P.learned_dims()
    rng = np.random.default_rng(21)
    th, flat = _params(rng, dm["n_in"], dm["n_out"])
    nw1 = mlp.HIDDEN * dm["n_in"] + mlp.HIDDEN
    flat[nw1:] = 0.0                              # start from the zero predictor
    P.learned_set_params(flat)
    N = P.level_size(0)
    Xs, Ts = [], []
    for seed in range(8):                       # seeded discrete forcings b = S x_true
        xt = np.random.default_rng(1000 + seed).standard_normal(N)
        X, T = P.learned_collect(torch.from_numpy(xt).cuda(), 3)
        Xs.append(X)
        Ts.append(T)
    X, T = torch.cat(Xs), torch.cat(Ts)
    hist = P.learned_train(X, T, steps=800, batch=1024, lr=1e-3, seed=7)
    zero = float(0.5 * (T.double() ** 2).sum(dim=1).mean())
    assert np.isfinite(hist).all()
    assert hist[-50:].mean() < 0.9 * zero, (zero, hist[-50:].mean())   # learned something beyond y = 0
    _, its0, h0, _, ok0 = P.solve()
    P.learned_enable(True)
    _, its1, h1, _, ok1 = P.solve()
    P.learned_enable(False)
    print(f"[gain] FGMRES its plain {its0} learned {its1}; loss {hist[:10].mean():.3e} -> {hist[-50:].mean():.3e}"
          f" (zero predictor {zero:.3e})")
    assert ok0 and ok1
    assert its1 <= its0
