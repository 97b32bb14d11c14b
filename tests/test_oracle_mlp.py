"""CPU pins of the learned smoother's reference network (oracle/mlp.py):
backpropagation against central finite differences of the loss, the first Adam
step against its closed form, the residual window on a hand-checked mesh, the
scale normalisation (positive homogeneity), and the minimal-residual step."""
import numpy as np

from oracle import mlp
from synth import cartesian_quads


def _net(rng, n_in, n_out):
    th = mlp.init_params(n_in, n_out, rng.random(mlp.HIDDEN * n_in), rng.random(n_out * mlp.HIDDEN))
    th["b1"] = 0.1 * rng.standard_normal(mlp.HIDDEN)
    th["b2"] = 0.1 * rng.standard_normal(n_out)
    return th


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    n_in, n_out, B = 9, 4, 7
    th = _net(rng, n_in, n_out)
    X, T = rng.standard_normal((B, n_in)), rng.standard_normal((B, n_out))
    _, g = mlp.loss_and_grad(th, X, T, quantize=False)
    h = 1e-6
    for k in th:
        flat = th[k].ravel()
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            tp = {q: v.copy() for q, v in th.items()}
            tm = {q: v.copy() for q, v in th.items()}
            tp[k].ravel()[idx] += h
            tm[k].ravel()[idx] -= h
            fd = (mlp.loss_and_grad(tp, X, T, quantize=False)[0] - mlp.loss_and_grad(tm, X, T, quantize=False)[0]) / (2 * h)
            assert abs(fd - g[k].ravel()[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx)


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(1)
    th = {"a": rng.standard_normal(5)}
    g = {"a": rng.standard_normal(5)}
    z = {"a": np.zeros(5)}
    lr = 1e-3
    th2, m2, v2 = mlp.adam_step(th, g, z, z, 1, lr)
    # m_hat = g, v_hat = g^2 after bias correction at step 1
    assert np.allclose(th2["a"], th["a"] - lr * g["a"] / (np.abs(g["a"]) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m2["a"], 0.1 * g["a"]) and np.allclose(v2["a"], 0.001 * g["a"] ** 2)


def test_window_of_interior_face():
    mesh = cartesian_quads(2)
    d, p, t = 2, 1, 1
    L = mlp.layout(mesh, d, p, t)
    assert L.Fm == 4 and L.n_res == 2 * (4 * 2 + 1) and L.n_in == L.n_res + 8
    r = np.arange(1, mesh.n_faces * d * p + mesh.n_cells * t + 1, dtype=float)
    X, s = mlp.windows(mesh, L, r)
    fc = mesh.face_cells()
    f = int(np.flatnonzero(fc[:, 1] >= 0)[0])
    c0, c1 = fc[f]
    raw = []
    for c in (c0, c1):
        for g in mesh.cell_faces(c):
            raw += list(r[g * 2:g * 2 + 2])
        raw += [r[L.nface + c]]
    raw = np.array(raw)
    assert np.isclose(s[f], np.sqrt(np.sum(raw ** 2) / L.n_res))
    assert np.allclose(X[f, :L.n_res] * s[f], raw)
    oh = X[f, L.n_res:]
    assert oh[list(mesh.cell_faces(c0)).index(f)] == 1 and oh[4 + list(mesh.cell_faces(c1)).index(f)] == 1
    assert oh.sum() == 2
    fb = int(np.flatnonzero(fc[:, 1] < 0)[0])           # boundary face: second side empty
    assert X[fb, L.n_res + 4:].sum() == 0 and np.all(X[fb, L.n_res // 2:L.n_res] == 0)


def test_correction_is_positively_homogeneous():
    rng = np.random.default_rng(2)
    mesh = cartesian_quads(3)
    L = mlp.layout(mesh, 2, 2, 3)
    th = _net(rng, L.n_in, L.n_out)
    r = rng.standard_normal(L.nface + mesh.n_cells * L.t)
    z1 = mlp.apply(th, mesh, L, r, quantize=False)
    z2 = mlp.apply(th, mesh, L, 7.5 * r, quantize=False)
    assert np.allclose(z2, 7.5 * z1, rtol=1e-12, atol=0)


def test_pressure_head_is_the_mean_over_the_cell_faces():
    """With W2 = 0 the outputs are b2: face blocks get s_F b2[:dp], and a cell
    the mean over its faces F of s_F times the b2 slice of its side of F."""
    rng = np.random.default_rng(5)
    mesh = cartesian_quads(2)
    L = mlp.layout(mesh, 2, 1, 2)
    th = _net(rng, L.n_in, L.n_out)
    th["W2"][:] = 0.0
    th["b2"] = np.arange(1.0, L.n_out + 1.0)         # [1, 2 | 3, 4 | 5, 6]
    r = rng.standard_normal(L.nface + mesh.n_cells * L.t)
    z = mlp.apply(th, mesh, L, r, quantize=False)
    _, s = mlp.windows(mesh, L, r)
    fc = mesh.face_cells()
    for f in range(mesh.n_faces):
        assert np.allclose(z[2 * f:2 * f + 2], s[f] * np.array([1.0, 2.0]))
    c = 0
    want = np.zeros(2)
    for f in mesh.cell_faces(c):
        want += s[f] * (np.array([3.0, 4.0]) if fc[f, 0] == c else np.array([5.0, 6.0]))
    assert np.allclose(z[L.nface:L.nface + 2], want / 4)


def test_targets_carry_face_and_both_cells():
    mesh = cartesian_quads(2)
    L = mlp.layout(mesh, 2, 1, 1)
    e = np.arange(1.0, L.nface + mesh.n_cells + 1.0)
    s = np.full(mesh.n_faces, 2.0)
    s[0] = 0.0
    T = mlp.targets(mesh, L, e, s)
    fc = mesh.face_cells()
    assert np.all(T[0] == 0)
    f = int(np.flatnonzero(fc[:, 1] >= 0)[0])
    assert np.allclose(T[f], np.array([e[2 * f], e[2 * f + 1], e[L.nface + fc[f, 0]], e[L.nface + fc[f, 1]]]) / 2)
    fb = int(np.flatnonzero((fc[:, 1] < 0) & (np.arange(mesh.n_faces) > 0))[0])
    assert T[fb, 3] == 0


def test_bfloat16_network_definition():
    """On values of the bfloat16 grid whose products and sums stay on it, the
    rounded network equals the unrounded one; on general values the two differ
    by the rounding of x, W1, W2 and h (2^-8 relative each)."""
    rng = np.random.default_rng(6)
    n_in, n_out, B = 8, 3, 5
    th = {"W1": rng.integers(-3, 4, (mlp.HIDDEN, n_in)).astype(float), "b1": np.zeros(mlp.HIDDEN),
          "W2": rng.integers(-3, 4, (n_out, mlp.HIDDEN)) / 4.0, "b2": np.full(n_out, 0.1)}
    X = rng.integers(-2, 3, (B, n_in)).astype(float)
    assert np.array_equal(mlp.forward(th, X, True)[0], mlp.forward(th, X, False)[0])
    th = _net(rng, n_in, n_out)
    X = rng.standard_normal((B, n_in))
    Yq, Y = mlp.forward(th, X, True)[0], mlp.forward(th, X, False)[0]
    assert 0 < np.abs(Yq - Y).max() <= 4 * 2.0 ** -8 * np.abs(Y).max() + 1e-3
    g_q = mlp.loss_and_grad(th, X, np.zeros((B, n_out)), True)[1]
    g = mlp.loss_and_grad(th, X, np.zeros((B, n_out)), False)[1]
    for k in g:
        assert np.abs(g_q[k] - g[k]).max() <= 0.05 * np.abs(g[k]).max() + 1e-12


def test_mr_step_minimises_over_directions():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((20, 20)) + 5 * np.eye(20)
    r = rng.standard_normal(20)
    dirs = [rng.standard_normal(20) for _ in range(3)]
    x = mlp.mr_step(lambda v: A @ v, dirs, np.zeros(20), r)
    x2 = mlp.mr_step(lambda v: A @ v, dirs[:2], np.zeros(20), r)
    assert np.linalg.norm(r - A @ x) <= np.linalg.norm(r - A @ x2) + 1e-14
    W = A @ np.stack(dirs, 1)
    y = np.linalg.solve(W.T @ W, W.T @ r)                 # normal equations give the same minimiser
    assert np.allclose(x, np.stack(dirs, 1) @ y)
