"""Host logic of the sparse direct coarse solver (options.coarse_mode = "direct";
the paper solves its 2D coarse problems directly, Section 5.2): the symbolic
phase's nested dissection, pressure placement and index maps, read back through
hho_direct_info, drive an independent NumPy elimination of the fronts in the
order the device uses (sweep operator on each front's own unknowns, updates
passed to the parent through the child maps, forward and backward passes).
That elimination must reproduce the bordered direct solution of the oracle's
coarsest operator (np.linalg.solve of [S z; z^T 0]) to rounding, which fails if
a front misses an unknown, a child map is wrong, an operator entry is assembled
into the wrong front or twice, or a pressure is eliminated before the velocity
unknowns that make its pivot nonzero (a zero pivot).  No GPU is used."""
import numpy as np
import pytest

from synth import voronoi_lloyd, polynomial_stokes, cartesian_quads, cartesian_hexes
from synth.fields import problem_data

NAMES = ["m", "nfs", "child", "dofoff", "dof", "cmap", "hptr", "hfront", "pinned", "sizes"]


def _eliminate(S, z, I, b, allow_missing=()):
    m, nfs, child, dofoff, dof, cmap = (I[n] for n in NAMES[:6])
    nn, N = len(m), S.shape[0]
    pinned = int(I["pinned"][0])
    # fronts are numbered children first; each eliminates its first nfs unknowns
    ekey = np.full(N, np.iinfo(np.int64).max)
    front_of = np.full(N, -1)
    key = 0
    for f in range(nn):
        own = dof[dofoff[f]:dofoff[f] + nfs[f]]
        ekey[own] = np.arange(key, key + nfs[f])
        front_of[own] = f
        key += nfs[f]
    assert key == N - (pinned >= 0) - len(allow_missing)
    assert (front_of >= 0).sum() == key and (pinned < 0 or front_of[pinned] < 0)
    assert all(front_of[i] < 0 for i in allow_missing)
    fronts = []
    for f in range(nn):
        d = dof[dofoff[f]:dofoff[f + 1]]
        assert len(set(d.tolist())) == m[f]
        # an operator entry belongs to the front of its earlier-eliminated unknown
        owner = np.where(ekey[d][:, None] < ekey[d][None, :], front_of[d][:, None], front_of[d][None, :])
        M = np.where(owner == f, S[np.ix_(d, d)], 0.0)
        for s in range(2):
            c = child[2 * f + s]
            if c < 0:
                continue
            cm = cmap[2 * dofoff[f]:2 * dofoff[f + 1]][s::2]
            idx = np.where(cm >= 0)[0]
            assert len(idx) == m[c] - nfs[c]          # every update of the child has a place
            U = fronts[c][nfs[c]:, nfs[c]:]
            M[np.ix_(idx, idx)] += U[np.ix_(cm[idx], cm[idx])]
        for k in range(nfs[f]):
            a = M[k, k]
            assert a != 0.0 and np.isfinite(a), (f, k)
            r, col = M[k, :].copy(), M[:, k].copy()
            M -= np.outer(col, r) / a
            M[k, :], M[:, k] = r / a, col / a
            M[k, k] = -1.0 / a
        fronts.append(M)
    coef = (z @ b) / (z @ z) if pinned >= 0 else 0.0
    bp = b - coef * z if pinned >= 0 else b
    V = []
    for f in range(nn):
        d = dof[dofoff[f]:dofoff[f + 1]]
        v = np.zeros(m[f])
        v[:nfs[f]] = bp[d[:nfs[f]]]
        for s in range(2):
            c = child[2 * f + s]
            if c >= 0:
                cm = cmap[2 * dofoff[f]:2 * dofoff[f + 1]][s::2]
                idx = np.where(cm >= 0)[0]
                v[idx] += V[c][nfs[c]:][cm[idx]]
        u = v.copy()
        u[nfs[f]:] -= fronts[f][nfs[f]:, :nfs[f]] @ v[:nfs[f]]
        V.append(u)
    x = np.zeros(N)
    for f in reversed(range(nn)):
        d = dof[dofoff[f]:dofoff[f + 1]]
        y = np.concatenate([V[f][:nfs[f]], x[d[nfs[f]:]]])
        x[d[:nfs[f]]] = -(fronts[f][:nfs[f], :] @ y)
    if pinned >= 0:
        x[pinned] = 0.0
        x -= (z @ x) / (z @ z) * z
    return x


def _eliminate_batch(S, zs, I, b):
    """The same for a batch: zs are the members' null vectors, one pinned
    unknown per member; b is made orthogonal to each, and so is x."""
    pins = [int(v) for v in I["pinned"]]
    assert len(pins) == len(zs) and all(v >= 0 for v in pins)
    bp = b.copy()
    for z in zs:
        bp -= (z @ bp) / (z @ z) * z
    I1 = dict(I)
    I1["pinned"] = np.array([-1])
    keep = np.ones(S.shape[0], bool)
    keep[pins] = False
    # eliminate with the pinned unknowns' rows and columns removed (they are in no front)
    x = _eliminate(np.where(np.outer(keep, keep), S, 0.0) + np.diag(~keep * 1.0), None, I1, bp, allow_missing=pins)
    x[pins] = 0.0
    for z in zs:
        x -= (z @ x) / (z @ z) * z
    return x


@pytest.mark.parametrize("name,mk,k,cond", [
    ("vor60_k2_v", lambda: voronoi_lloyd(60, 2), 2, "v"),
    ("vor60_k2_vp", lambda: voronoi_lloyd(60, 2), 2, "vp"),
    ("vor200_k3_v", lambda: voronoi_lloyd(200, 5), 3, "v"),
    ("quad6_k1_v_neumann", lambda: cartesian_quads(6).with_bc(lambda x: 2 if x[0] > 1 - 1e-12 else 1), 1, "v"),
    ("hex3_k1_vp", lambda: cartesian_hexes(3), 1, "vp"),
    ("hex4_k1_v", lambda: cartesian_hexes(4), 1, "v"),
])
def test_fronts_reproduce_the_bordered_direct_solution(name, mk, k, cond):
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    mesh = mk()
    data = problem_data(polynomial_stokes(mesh.dim, k + 1, 3), None, mesh.dim)
    P = H.Problem(H.Mesh(mesh), k, cond, coarse_mode="direct")
    P.set_data(*data)
    I = {n: P.direct_info(n) for n in NAMES}
    O = OS.build(mesh, k, cond, data, eta=None)
    S, z = O.S[-1].toarray(), O.z[-1]
    N = S.shape[0]
    b = np.random.default_rng(1).standard_normal(N)
    x = _eliminate(S, z, I, b)
    if z is not None:
        xd = np.linalg.solve(np.block([[S, z[:, None]], [z[None, :], np.zeros((1, 1))]]), np.append(b, 0.0))[:N]
        assert I["pinned"][0] >= 0
    else:
        xd = np.linalg.solve(S, b)
        assert I["pinned"][0] < 0
    err = np.abs(x - xd).max() / np.abs(xd).max()
    nfront, nheight = I["sizes"][:2]
    print(f"[direct symbolic] {name}: {N} unknowns, {nfront} fronts, {nheight} heights, err {err:.1e}")
    assert nheight >= 2 and err <= 1e-11


@pytest.mark.parametrize("name,mk,k,cond", [
    ("quad1_k1_v", lambda: cartesian_quads(1), 1, "v"),
    ("quad1_k2_vp", lambda: cartesian_quads(1), 2, "vp"),
    ("hex1_k1_v", lambda: cartesian_hexes(1), 1, "v"),
    ("quad1_k1_v_neumann", lambda: cartesian_quads(1).with_bc(lambda x: 2 if x[0] > 1 - 1e-12 else 1), 1, "v"),
])
def test_one_cell_is_one_front(name, mk, k, cond):
    """Degenerate input: a single cell is one leaf front that eliminates all it
    holds: every unknown, except, with the constant-pressure null space, the
    cell's one pressure, which is the pinned unknown (in no front); without it (a
    Neumann side) nothing is pinned."""
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    mesh = mk()
    data = problem_data(polynomial_stokes(mesh.dim, k + 1, 3), None, mesh.dim)
    P = H.Problem(H.Mesh(mesh), k, cond, coarse_mode="direct")
    P.set_data(*data)
    I = {n: P.direct_info(n) for n in NAMES}
    O = OS.build(mesh, k, cond, data, eta=None)
    S, z = O.S[-1].toarray(), O.z[-1]
    N = S.shape[0]
    assert list(I["sizes"][:2]) == [1, 1]
    assert I["m"][0] == I["nfs"][0] == N - (z is not None)
    assert (I["pinned"][0] == N - 1) if z is not None else (I["pinned"][0] < 0)
    b = np.random.default_rng(4).standard_normal(N)
    x = _eliminate(S, z, I, b)
    if z is not None:
        xd = np.linalg.solve(np.block([[S, z[:, None]], [z[None, :], np.zeros((1, 1))]]), np.append(b, 0.0))[:N]
    else:
        xd = np.linalg.solve(S, b)
    assert np.abs(x - xd).max() <= 1e-12 * np.abs(xd).max()


def test_direct_mode_rejects_what_it_cannot_solve():
    import paper_2009_13840_amd as H
    with pytest.raises(H.HHOError):
        H.Problem(H.Mesh(cartesian_quads(2)), 1, "v", coarse_mode="direct", degrees=[1])  # coarsest degree 1
    with pytest.raises(H.HHOError):
        H.Problem(H.Mesh(cartesian_quads(2)), 1, "v", coarse_mode=5)                     # no such solver
    P = H.Problem(H.Mesh(cartesian_quads(4)), 1, "v", coarse_mode="direct")
    with pytest.raises(H.HHOError):
        P.direct_info("m")                                                               # before set_data
    P.set_data(*problem_data(polynomial_stokes(2, 2, 3), None, 2))
    with pytest.raises(H.HHOError):
        P.direct_info("no such array")


def test_batch_fronts_pin_one_pressure_per_member():
    """A batch of pure-Dirichlet members (disjoint union): the symbolic phase
    leaves one pressure per member at the root and pins it; the elimination with
    per-member projections reproduces each member's bordered direct solution."""
    import scipy.sparse as sp
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    from synth.batch import shifted, region_fields
    members = [voronoi_lloyd(40, 3), cartesian_quads(5), voronoi_lloyd(25, 6)]
    k, cond, width = 2, "v", 2.0
    fields = [problem_data(polynomial_stokes(2, k + 1, 50 + i), None, 2) for i in range(len(members))]
    U, fo, co = H.Mesh.union([shifted(m, width * i) for i, m in enumerate(members)])
    P = H.Problem(U, k, cond, coarse_mode="direct")
    P.set_segments(fo, co)
    P.set_data(*region_fields(fields, 2, width))
    I = {n: P.direct_info(n) for n in NAMES}
    assert len(I["pinned"]) == len(members)
    # the union's coarsest operator from the members' own (block diagonal, union layout)
    Os = [OS.build(m, k, cond, f, eta=None) for m, f in zip(members, fields)]
    dp = Os[0].lays[-1].off // members[0].n_faces     # face unknowns per face on the coarsest level
    nface = int(fo[-1]) * dp
    N = nface + int(co[-1])
    S = np.zeros((N, N))
    zs = []
    for i, O in enumerate(Os):
        Si, nf_i = O.S[-1].toarray(), O.lays[-1].off
        idx = np.concatenate([np.arange(fo[i] * dp, fo[i] * dp + nf_i), nface + np.arange(co[i], co[i + 1])])
        S[np.ix_(idx, idx)] = Si
        z = np.zeros(N)
        z[idx] = O.z[-1]
        zs.append(z)
    b = np.random.default_rng(2).standard_normal(N)
    x = _eliminate_batch(S, zs, I, b)
    for i, O in enumerate(Os):
        Si, z, nf_i = O.S[-1].toarray(), O.z[-1], O.lays[-1].off
        idx = np.concatenate([np.arange(fo[i] * dp, fo[i] * dp + nf_i), nface + np.arange(co[i], co[i + 1])])
        n = len(idx)
        xd = np.linalg.solve(np.block([[Si, z[:, None]], [z[None, :], np.zeros((1, 1))]]), np.append(b[idx], 0.0))[:n]
        err = np.abs(x[idx] - xd).max() / np.abs(xd).max()
        print(f"[direct symbolic batch] member {i}: err {err:.1e}")
        assert err <= 1e-11
