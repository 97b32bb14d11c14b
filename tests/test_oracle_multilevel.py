"""Pins of the oracle's smoother preconditioners, V-cycle composition and coarse
block preconditioner (Section 3.3; Section 5.2 solver options).  CPU only.

Each pin is a property the definitions fix independently of how the oracle
evaluates them:

* cell-patch Schwarz: the weights form a partition of unity; on one cell, and
  on cells that share no face, it is the exact inverse;
* V-cycle: without smoothing it is the Galerkin coarse correction P S_c^-1 P^T;
  with exact smoothers it is S^-1; with one minimal-residual step per smoothing
  (identity preconditioner) it is the closed-form composition of the textbook
  minimal-residual iteration and the coarse correction;
* block-triangular coarse preconditioner: with an exact velocity solve it is the
  inverse of the upper block-triangular matrix [[A, C], [0, -S_d]]; with an
  exact (diagonal) Schur complement the preconditioned saddle-point matrix K
  satisfies (K P^-1 - I)^2 = 0, so GMRES ends in two iterations;
* smoothed-aggregation V-cycle: symmetric positive definite for an SPD matrix
  (symmetric smoothing), and on two levels equal to the two-grid error
  propagation formula;
* zero-fill ILU: L U equals A on A's pattern; with no fill possible (tridiagonal
  or dense pattern) it is the exact LU factorisation.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from synth import cartesian_quads, voronoi_lloyd, cartesian_hexes, polynomial_stokes, trig_series
from synth.batch import disjoint_union, shifted
from synth.fields import problem_data
import oracle.solve as OS
from oracle.multilevel import Schwarz
from oracle.system import prolongation
from oracle.krylov import gmres_solve
from oracle import amg as AM
from oracle.ilu import ILU0


def _neumann_right(mesh, x1=1.0):
    return mesh.with_bc(lambda x: 2 if x[0] > x1 - 1e-12 else 1)


def _build(mesh, k, cond, seed=3):
    return OS.build(mesh, k, cond, problem_data(None, trig_series(mesh.dim, seed), mesh.dim))


# ---------------------------------------------------------------- Schwarz

@pytest.mark.parametrize("mk,k,cond", [(lambda: voronoi_lloyd(20, 3), 2, "v"), (lambda: voronoi_lloyd(20, 3), 2, "vp"),
                                       (lambda: cartesian_hexes(2), 1, "v"), (lambda: cartesian_hexes(2), 1, "vp")])
def test_schwarz_weights_are_a_partition_of_unity(mk, k, cond):
    """The corrections of the patches sharing an unknown add up with weights
    summing to one (1/card(T_F) on face unknowns, 1 on a cell's pressure)."""
    mesh = mk()
    P = _build(mesh, k, cond)
    for l, S in enumerate(P.S):
        M = Schwarz(S, mesh, P.lays[l])
        tot = np.zeros(S.shape[0])
        cover = np.zeros(S.shape[0], dtype=int)
        for idx, w in zip(M.patches, M.weights):
            np.add.at(tot, idx, w)
            np.add.at(cover, idx, 1)
        assert np.all(cover >= 1)
        assert np.abs(tot - 1.0).max() < 1e-15


@pytest.mark.parametrize("dim,k,cond", [(2, 2, "v"), (2, 2, "vp"), (2, 3, "v"), (3, 1, "v"), (3, 1, "vp")])
def test_schwarz_on_one_cell_is_the_inverse(dim, k, cond):
    """One cell (a Neumann face removes the pressure null space): its patch is the
    whole system and the preconditioner is S^-1."""
    mesh = _neumann_right(cartesian_quads(1) if dim == 2 else cartesian_hexes(1))
    P = _build(mesh, k, cond)
    S = P.S[0]
    M = Schwarz(S, mesh, P.lays[0])
    r = np.random.default_rng(0).standard_normal(S.shape[0])
    x = spla.spsolve(S.tocsc(), r)
    assert np.abs(M(r) - x).max() < 1e-11 * np.abs(x).max()


@pytest.mark.parametrize("cond", ["v", "vp"])
def test_schwarz_on_unconnected_cells_is_the_inverse(cond):
    """Cells that share no face make S block diagonal by patches: every patch
    solve is exact and the preconditioner is S^-1 on every level."""
    cells = [_neumann_right(shifted(cartesian_quads(1), 2.0 * i), 2.0 * i + 1.0) for i in range(3)]
    mesh = disjoint_union(cells)
    P = _build(mesh, 2, cond)
    rng = np.random.default_rng(1)
    for l, S in enumerate(P.S):
        M = Schwarz(S, mesh, P.lays[l])
        r = rng.standard_normal(S.shape[0])
        x = spla.spsolve(S.tocsc(), r)
        assert np.abs(M(r) - x).max() < 1e-11 * np.abs(x).max(), l


# ---------------------------------------------------------------- V-cycle

def _prolongations(P):
    return [prolongation(P.lays[l], P.lays[l + 1]) for l in range(len(P.lays) - 1)]


@pytest.mark.parametrize("cond", ["v", "vp"])
def test_vcycle_without_smoothing_is_the_galerkin_coarse_correction(cond):
    """With no smoothing iterations the V-cycle is P_0 ... P_{L-1} S_L^-1
    P_{L-1}^T ... P_0^T b (restriction of the defect, coarse solve, prolongation)."""
    mesh = _neumann_right(voronoi_lloyd(16, 5))
    P = _build(mesh, 2, cond)
    H = OS.hierarchy(P, smooth_its=0, coarse="direct")
    Ps = _prolongations(P)
    b = np.random.default_rng(2).standard_normal(P.S[0].shape[0])
    R = b
    for Pl in Ps:
        R = Pl.T @ R
    c = spla.spsolve(P.S[-1].tocsc(), R)
    for Pl in reversed(Ps):
        c = Pl @ c
    x = H.vcycle(0, b)
    assert np.abs(x - c).max() < 1e-12 * np.abs(c).max()


@pytest.mark.parametrize("cond", ["v", "vp"])
def test_vcycle_with_exact_smoothers_is_exact(cond):
    mesh = _neumann_right(voronoi_lloyd(16, 6))
    P = _build(mesh, 2, cond)
    H = OS.hierarchy(P, coarse="direct")
    H.prec = [(lambda S: (lambda r: spla.spsolve(S.tocsc(), r)))(S) for S in P.S]
    b = np.random.default_rng(3).standard_normal(P.S[0].shape[0])
    x = spla.spsolve(P.S[0].tocsc(), b)
    assert np.abs(H.vcycle(0, b) - x).max() < 1e-10 * np.abs(x).max()


@pytest.mark.parametrize("cond,nlev", [("v", 2), ("vp", 2), ("v", 3)])
def test_vcycle_with_minimal_residual_smoothing(cond, nlev):
    """One right-preconditioned GMRES iteration with the identity preconditioner is
    the minimal-residual step w + a r, a = (S r, r) / (S r, S r).  The V-cycle of
    Section 3.3 is then, written out: pre-smoothing step from w = 0, defect
    restriction, recursion (coarsest: direct solve), prolongation of the
    correction, post-smoothing step."""
    mesh = _neumann_right(voronoi_lloyd(18, 7))
    k = nlev - 1
    P = _build(mesh, k, cond)
    H = OS.hierarchy(P, smooth_its=1, coarse="direct")
    H.prec = [lambda r: r.copy() for _ in P.S]
    Ps = _prolongations(P)

    def mr(S, b, w):
        r = b - S @ w
        Sr = S @ r
        return w + (Sr @ r) / (Sr @ Sr) * r

    def V(l, b):
        S = P.S[l]
        w = mr(S, b, np.zeros_like(b))
        d = Ps[l].T @ (b - S @ w)
        c = spla.spsolve(P.S[l + 1].tocsc(), d) if l + 1 == len(P.S) - 1 else V(l + 1, d)
        w = w + Ps[l] @ c
        return mr(S, b, w)

    b = np.random.default_rng(4).standard_normal(P.S[0].shape[0])
    x = V(0, b)
    assert np.abs(H.vcycle(0, b) - x).max() < 1e-11 * np.abs(x).max()


# ---------------------------------------------------------------- coarse block preconditioner

def _coarse_k0(mesh, cond="v"):
    P = _build(mesh, 0, cond)
    return P.S[0], P.lays[0]


def test_block_preconditioner_with_exact_velocity_solve():
    """On a coarsest level of at most 128 faces the AMG hierarchy is a dense
    inverse, so the velocity solve is exact (the v-cond k = 0 velocity block is
    s (x) I_d): the preconditioner is the inverse of [[A, C], [0, -diag(S_d)]]."""
    mesh = voronoi_lloyd(20, 8)
    S, lay = _coarse_k0(mesh)
    nf = lay.off
    Bp = AM.BlockStokesPrec(S, nf, mesh.dim)
    assert Bp.amg.Ainv is not None and not Bp.amg.levels
    Sd_ = S.toarray()
    A, C = Sd_[:nf, :nf], Sd_[:nf, nf:]
    # the velocity block is s (x) I_d: the components do not couple
    for c in range(mesh.dim):
        for c2 in range(mesh.dim):
            if c != c2:
                assert np.abs(A[c::mesh.dim, c2::mesh.dim]).max() == 0.0
    T = np.block([[A, C], [np.zeros((S.shape[0] - nf, nf)), -np.diag(Bp.Sd)]])
    v = np.random.default_rng(5).standard_normal(S.shape[0])
    z = Bp(v)
    zt = np.linalg.solve(T, v)
    assert np.abs(z - zt).max() < 1e-11 * np.abs(zt).max()


def test_block_preconditioner_with_exact_schur_complement_converges_in_two():
    """Saddle-point K = [[A, C], [C^T, 0]] with diagonal A = s (x) I_d and pressures
    coupled to disjoint velocity unknowns: C^T A^-1 C is diagonal and equals the
    preconditioner's S_d, so K P^-1 = [[I, 0], [C^T A^-1, I]] and GMRES with it
    converges in two iterations (minimal polynomial (t - 1)^2)."""
    rng = np.random.default_rng(6)
    d, nfaces, npres = 2, 40, 12
    s = 1.0 + rng.random(nfaces)
    A = np.kron(np.diag(s), np.eye(d))
    nfd = nfaces * d
    C = np.zeros((nfd, npres))
    perm = rng.permutation(nfd)
    for q in range(npres):
        rows = perm[q * 5:(q + 1) * 5]          # 5 velocity unknowns per pressure, disjoint
        C[rows, q] = rng.standard_normal(5)
    K = np.block([[A, C], [C.T, np.zeros((npres, npres))]])
    Ks = sp.csr_matrix(K)
    Bp = AM.BlockStokesPrec(Ks, nfd, d)
    assert np.allclose(Bp.Sd, np.diag(C.T @ np.linalg.solve(A, C)), rtol=1e-13, atol=0)
    n = K.shape[0]
    Pinv = np.stack([Bp(e) for e in np.eye(n)], axis=1)
    E = K @ Pinv - np.eye(n)
    assert np.abs(E @ E).max() < 1e-12 * np.abs(K).max()
    b = rng.standard_normal(n)
    x, its = gmres_solve(lambda v: K @ v, Bp, b, 1e-12, 30, 30)
    assert its <= 2
    assert np.linalg.norm(K @ x - b) < 1e-10 * np.linalg.norm(b)


# ---------------------------------------------------------------- smoothed aggregation

def _poisson(n):
    T = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    I = sp.eye(n)
    return (sp.kron(T, I) + sp.kron(I, T)).tocsr()


def test_sa_vcycle_is_symmetric_positive_definite():
    """Damped Jacobi before and after the coarse correction, same sweep count:
    the V-cycle operator B is symmetric, and positive definite for SPD A."""
    A = _poisson(20)                               # 400 rows: two or more levels
    S = AM.SA(A)
    assert len(S.levels) >= 1
    n = A.shape[0]
    B = np.stack([S.vcycle(e) for e in np.eye(n)], axis=1)
    assert np.abs(B - B.T).max() < 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_sa_two_level_error_propagation():
    """On two levels with an exact coarse solve the V-cycle's error propagation is
    I - B A = (I - w D^-1 A)^nu (I - P A_c^-1 P^T A) (I - w D^-1 A)^nu,
    w = 4 / (3 lambda)."""
    A = _poisson(14)                               # 196 rows -> one coarse level <= 128
    S = AM.SA(A, nu=2)
    assert len(S.levels) == 1 and S.Ainv is not None
    A0, P, Di = S.levels[0]
    n = A.shape[0]
    Ad, Pd = A0.toarray(), P.toarray()
    w = 4.0 / (3.0 * S.lams[0])
    Sm = np.eye(n) - w * np.diag(Di) @ Ad
    Ac = Pd.T @ Ad @ Pd
    Cc = np.eye(n) - Pd @ np.linalg.solve(Ac, Pd.T @ Ad)
    E = np.linalg.matrix_power(Sm, 2) @ Cc @ np.linalg.matrix_power(Sm, 2)
    B = np.stack([S.vcycle(e) for e in np.eye(n)], axis=1)
    assert np.abs((np.eye(n) - B @ Ad) - E).max() < 1e-11


# ---------------------------------------------------------------- zero-fill ILU

@pytest.mark.parametrize("mk,k,cond", [(lambda: voronoi_lloyd(12, 9), 2, "v"), (lambda: voronoi_lloyd(12, 9), 2, "vp"),
                                       (lambda: cartesian_hexes(2), 1, "v")])
def test_ilu0_matches_a_on_its_pattern(mk, k, cond):
    """(L U)_ij = a_ij for every (i, j) of A's pattern, L unit lower, U upper."""
    P = _build(mk(), k, cond)
    for S in P.S:
        F = ILU0(S)
        LU = (F.L @ F.U).tocsr()
        S = sp.csr_matrix(S)
        rows = np.repeat(np.arange(S.shape[0]), np.diff(S.indptr))
        diff = np.asarray(LU[rows, S.indices]).ravel() - S.data
        assert np.abs(diff).max() < 1e-11 * np.abs(S.data).max()
        assert np.all(F.L.diagonal() == 1.0)
        assert sp.triu(F.L, k=1).nnz == 0 and sp.tril(F.U, k=-1).nnz == 0


def test_ilu0_is_exact_lu_without_fill():
    """A tridiagonal matrix, and a matrix with a full pattern, have no fill
    outside their pattern: zero-fill ILU is their LU factorisation
    (symmetric and diagonally dominant, so partial pivoting swaps no rows)."""
    rng = np.random.default_rng(10)
    n = 30
    off = rng.uniform(-1, 1, n - 1)
    T = np.diag(3 + rng.random(n)) + np.diag(off, 1) + np.diag(off, -1)
    Dm = rng.uniform(-1, 1, (12, 12))
    Dm = Dm + Dm.T + 30 * np.eye(12)
    for M in (T, Dm):
        Pm, L, U = sla.lu(M)
        assert np.array_equal(Pm, np.eye(M.shape[0]))
        F = ILU0(sp.csr_matrix(M) if M is Dm else sp.csr_matrix(np.where(M != 0, M, 0.0)))
        assert np.abs(F.L.toarray() - L).max() < 1e-13
        assert np.abs(F.U.toarray() - U).max() < 1e-12 * np.abs(U).max()
        r = rng.standard_normal(M.shape[0])
        assert np.abs(F(r) - np.linalg.solve(M, r)).max() < 1e-12 * np.abs(np.linalg.solve(M, r)).max()


@pytest.mark.parametrize("cond", ["v", "vp"])
def test_fgmres_with_ilu_smoother_reaches_the_direct_solution(cond):
    """The paper's smoother (two ILU(0)-preconditioned GMRES iterations) inside the
    V-cycle: FGMRES reaches the direct solution."""
    mesh = voronoi_lloyd(24, 11)
    P = _build(mesh, 2, cond)
    x, its, hist, conv = OS.solve_fgmres(P, rtol=1e-10, smoother="ilu", coarse="direct")
    xd = OS.normalise_pressure(P, OS.solve_direct(P))
    assert conv and np.linalg.norm(x - xd) < 1e-8 * np.linalg.norm(xd)
    assert its <= 30


# ---------------------------------------------------------------- float32 emulation of the V-cycle

@pytest.mark.parametrize("cond", ["v", "vp"])
def test_fp32_vcycle_emulation_is_float32_and_close(cond):
    """The float32 emulation keeps float32 data above the coarsest level, and its
    V-cycle lies within the float32 rounding bound (1e-5 of the largest entry) of
    the FP64 V-cycle while differing from it (by more than 1e-9)."""
    from oracle.mixed import Vcycle32
    mesh = voronoi_lloyd(30, 12)
    P = _build(mesh, 2, cond)
    H = OS.hierarchy(P, coarse="direct")
    V32 = Vcycle32(H)
    assert all(S.dtype == np.float32 for S in V32.S)
    assert all(A.dtype == np.float32 for M in V32.prec for A in M.inv)
    b = OS.project_out(P.z[0])(np.random.default_rng(13).standard_normal(P.S[0].shape[0]))
    x64 = OS.project_out(P.z[0])(H.vcycle(0, b))
    x32 = OS.project_out(P.z[0])(V32(b))
    err = np.abs(x32 - x64).max() / np.abs(x64).max()
    assert 1e-9 < err < 1e-5, err


def test_one_level_vcycle_is_the_coarsest_solve():
    """With a single level (k = 0, no coarser degree) the V-cycle is the coarsest
    solve itself; FGMRES preconditioned by it converges at once."""
    mesh = _neumann_right(voronoi_lloyd(16, 14))
    P = _build(mesh, 0, "v")
    assert len(P.S) == 1
    H = OS.hierarchy(P, coarse="direct")
    b = np.random.default_rng(15).standard_normal(P.S[0].shape[0])
    x = spla.spsolve(P.S[0].tocsc(), b)
    assert np.abs(H.vcycle(0, b) - x).max() < 1e-12 * np.abs(x).max()
    xs, its, hist, conv = OS.solve_fgmres(P, rtol=1e-12, coarse="direct")
    assert conv and its == 1


def test_bfloat16_rounding_definition():
    """round_bf16 against values fixed by the definition of round-to-nearest-even
    on the bfloat16 grid (8 significand bits) and against a brute-force nearest
    search on random float32 values."""
    import numpy as np
    from oracle.mixed import round_bf16
    u = 2.0 ** -7                       # bfloat16 spacing on [1, 2)
    cases = {1.0: 1.0, 1.0 + u: 1.0 + u, 1.0 + u / 2: 1.0,                 # tie -> even (1.0)
             1.0 + 3 * u / 2: 1.0 + 2 * u,                                  # tie -> even (1 + 2u)
             1.0 + u / 2 + 2.0 ** -20: 1.0 + u, -(1.0 + 3 * u / 2): -(1.0 + 2 * u),
             2.0 ** -130: 2.0 ** -130, 0.0: 0.0, 3.0: 3.0, 1e38: None}
    for x, want in cases.items():
        got = float(round_bf16(np.float32(x)))
        if want is None:
            assert np.isfinite(got) and abs(got - 1e38) <= 2.0 ** -8 * 1e38
        else:
            assert got == want, (x, got, want)
    assert np.isnan(round_bf16(np.float32(np.nan)))
    assert round_bf16(np.float32(np.inf)) == np.inf
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-6, 6, 20000)).astype(np.float32)
    r = round_bf16(x)
    assert np.array_equal(round_bf16(r), r)                        # idempotent
    assert np.all((r.view(np.uint32) & 0xFFFF) == 0)               # on the bfloat16 grid
    # nearest of the grid neighbours (brute force over the two candidates)
    e = np.floor(np.log2(np.abs(x.astype(np.float64))))
    step = 2.0 ** (e - 7)
    lo = np.trunc(x.astype(np.float64) / step) * step
    hi = lo + np.sign(x) * step
    d_lo, d_hi = np.abs(x - lo), np.abs(x - hi)
    best = np.where(d_lo < d_hi, lo, hi)
    ties = d_lo == d_hi
    assert np.array_equal(r[~ties].astype(np.float64), best[~ties])


def test_product_copy_block_is_the_schur_complement_up_to_rounding():
    """The product copy's face block, with the bfloat16 rounding removed, is the
    face block of the Schur complement of eqs. ST.1 / ST.2 (checked against the
    oracle's dense-solve condensation), and with it differs by at most the
    rounding of its factors."""
    import numpy as np
    from unittest import mock
    import oracle.mixed as MX
    import oracle.solve as OS
    from oracle.condense import condense_v, condense_vp
    from synth import voronoi_lloyd, cartesian_hexes, polynomial_stokes
    from synth.fields import problem_data
    for mesh, k in ((voronoi_lloyd(12, 2), 2), (cartesian_hexes(1), 2)):
        data = problem_data(polynomial_stokes(mesh.dim, k + 1, 1), None, mesh.dim)
        P = OS.build(mesh, k, "v", data)
        for cond, cfun in (("v", condense_v), ("vp", condense_vp)):
            for L in P.locs[:4]:
                S = cfun(L)[0]
                n = L.nfaces * L.d * L.nF
                exact = S[:n, :n]
                with mock.patch.object(MX, "round_bf16", lambda a: np.asarray(a, dtype=np.float64)), \
                        mock.patch.object(MX, "F32", np.float64):
                    blk, _ = MX.product_copy_block(L, cond)
                assert np.abs(blk - exact).max() <= 1e-11 * np.abs(exact).max()
                blk16, bound = MX.product_copy_block(L, cond)
                err = np.abs(blk16 - exact)
                assert err.max() > 0
                assert np.all(err <= 2.0 ** -7 * (bound + np.abs(exact)) + 1e-12 * np.abs(exact).max())
