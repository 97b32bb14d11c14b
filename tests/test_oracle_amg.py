"""CPU pins of the coarsest-level smoothed-aggregation preconditioner of the
oracle (oracle/amg.py).  The AMG iterate has no closed form; these tests pin
what its definition fixes: aggregates partition the nodes around a root, the
spectral estimate brackets rho(D^{-1} A), coarsening stops before a nearly
dense level, and the V-cycle is a contraction on model Poisson matrices."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import amg as AM


def poisson(n, dim):
    T = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    I = sp.eye(n)
    if dim == 2:
        return (sp.kron(T, I) + sp.kron(I, T)).tocsr()
    return (sp.kron(sp.kron(T, I), I) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(I, I), T)).tocsr()


def test_aggregates_partition_around_a_root():
    A = poisson(20, 2)
    agg = AM.aggregate(A)
    assert agg.min() == 0 and set(np.unique(agg)) == set(range(agg.max() + 1))
    for a in range(agg.max() + 1):
        members = np.flatnonzero(agg == a)
        root = members.min()                       # the root opens its aggregate first
        nb = set(A.indices[A.indptr[root]:A.indptr[root + 1]]) | {root}
        assert set(members) <= nb


def test_spectral_estimate_brackets_rho():
    for A in (poisson(30, 2), poisson(12, 3)):
        D = A.diagonal()
        rho = abs(spla.eigs(sp.diags(1 / D) @ A, k=1, which="LM", return_eigenvectors=False)[0])
        lam = AM.spectral_radius_estimate(A)
        assert 0.95 * rho <= lam <= AM.LAMBDA_SAFETY * rho * (1 + 1e-12)


def test_density_stop_and_sweep_coarsest():
    A = poisson(16, 3)
    S = AM.SA(A)
    for Al, _, _ in S.levels[1:]:
        assert Al.nnz <= AM.MAX_ROW_NNZ * Al.shape[0]
    if S.Ac.shape[0] > AM.COARSEST:
        assert S.Ainv is None                      # Jacobi sweeps on a large coarsest level
    else:
        assert S.Ainv is not None


def _contraction(A, S, reps=6, seed=0):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(A.shape[0])
    an = lambda v: np.sqrt(v @ (A @ v))
    e0 = an(e)
    for _ in range(reps):
        e = e - S.vcycle(A @ e)
    return (an(e) / e0) ** (1.0 / reps)


def test_vcycle_contracts_on_poisson():
    for A, bound in ((poisson(48, 2), 0.3), (poisson(16, 3), 0.35)):
        for p_steps in (1, 2):
            S = AM.SA(A, p_steps=p_steps)
            assert len(S.levels) >= 1
            assert _contraction(A, S) < bound, p_steps


def test_second_smoothing_step_strengthens_the_cycle():
    """A second prolongator smoothing step widens P by one ring of neighbours
    (structurally, P_2 = pattern of P_1 + A P_1) and contracts faster on the 2D
    model problem."""
    A = poisson(48, 2)
    S1, S2 = AM.SA(A, p_steps=1), AM.SA(A, p_steps=2)
    assert S2.steps[0] == 2 and S1.steps[0] == 1
    P1, P2 = S1.levels[0][1], S2.levels[0][1]
    Ab = A.copy()
    Ab.data[:] = 1.0
    P1b = P1.copy()
    P1b.data[:] = 1.0
    pat = (P1b + Ab @ P1b).tocsr()
    pat.data[:] = 1.0
    P2b = P2.copy()
    P2b.eliminate_zeros()
    P2b.data[:] = 1.0
    outside = (P2b - P2b.multiply(pat)).tocsr()
    outside.eliminate_zeros()
    assert outside.nnz == 0                     # P_2 lies within the widened pattern
    assert P2b.nnz > P1.nnz
    assert _contraction(A, S2) < _contraction(A, S1)


def test_smoothing_steps_fall_back_before_a_dense_level():
    """On 3D grids two smoothing steps would make the next operator too dense:
    the level takes one step instead of stopping the coarsening."""
    A = poisson(16, 3)
    S = AM.SA(A, p_steps=2)
    for Al, _, _ in S.levels[1:]:
        assert Al.nnz <= AM.MAX_ROW_NNZ * Al.shape[0]
    assert all(st in (1, 2) for st in S.steps)
    assert len(S.levels) >= 1
