"""GPU tests of the V-cycle with reduced-precision storage (HHO_PREC_BF16 and
HHO_PREC_FP32) through the C ABI.

* The level operators in the V-cycle's storage against the oracle's operator
  with every value rounded the same way (FP64 -> float32, then to the nearest
  bfloat16, ties to even: oracle.mixed.round_bf16) applied to the float32-rounded
  input in exact arithmetic: the only difference left is the float32
  accumulation, bounded entry by entry by 1e-5 * (|S_r| |x_r|).
* The smoother preconditioner of the 16-bit mode keeps FP32 factors: for
  v&p-cond it equals the FP32 mode's exactly; for v-cond it also reads the
  operator's cell coupling, stored in 16 bits, so it agrees with the FP64 one to
  a few parts in a thousand (each value rounded by at most 2^-9; bound 3e-2 of
  the largest entry).  The FP32 one agrees with FP64 to FP32 rounding.
* FGMRES preconditioned by the bfloat16 V-cycle still reaches the FP64 true
  residual and the oracle's direct solution (P12: the outer solve is FP64).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from synth import cartesian_quads, voronoi_lloyd, cartesian_hexes, polynomial_stokes  # noqa: E402
from synth.fields import problem_data  # noqa: E402

CASES = [
    ("vor40_k3_v", lambda: voronoi_lloyd(40, 3), 3, "v"),
    ("quad4_k2_vp", lambda: cartesian_quads(4), 2, "vp"),
    ("hex2_k3_vp", lambda: cartesian_hexes(2), 3, "vp"),
    ("hex2_k2_v", lambda: cartesian_hexes(2), 2, "v"),
]


@pytest.fixture(scope="module")
def built():
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    cache = {}

    def get(name, mk, k, cond, precision):
        key = (name, precision)
        if key not in cache:
            mesh = mk()
            data = problem_data(polynomial_stokes(mesh.dim, k + 1, 3), None, mesh.dim)
            print(f"[case] {name} k={k} cond={cond} precision={precision}", flush=True)
            P = H.Problem(H.Mesh(mesh), k, cond, precision=precision, coarse_mode="dense", rtol=1e-10)
            P.set_data(*data)
            P.bind("cuda:0")
            P.setup()
            O = OS.build(mesh, k, cond, data, eta=None)
            cache[key] = (mesh, P, O)
        return cache[key]
    return get


def _rounded(S, precision):
    from oracle.mixed import round_bf16
    R = S.copy().astype(np.float64).tocsr()
    v = R.data.astype(np.float32)
    R.data = (round_bf16(v) if precision == "bf16" else v).astype(np.float64)
    return R


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
@pytest.mark.parametrize("name,mk,k,cond", CASES)
def test_vcycle_storage_operator_matches_rounded_oracle_operator(built, name, mk, k, cond, precision):
    import torch
    mesh, P, O = built(name, mk, k, cond, precision)
    rng = np.random.default_rng(31)
    for l in range(len(O.S) - 1):          # levels above the coarsest run in reduced precision
        S = O.S[l]
        x = rng.standard_normal(S.shape[0])
        x32 = x.astype(np.float32).astype(np.float64)
        Sr = _rounded(S, precision)
        want = Sr @ x32
        bound = abs(Sr) @ np.abs(x32)
        got = P.vcycle_level_apply(l, torch.from_numpy(x).cuda()).cpu().numpy()
        excess = np.abs(got - want) - 1e-5 * bound
        print(f"[{precision} operator] {name} level {l}: max |err| / bound "
              f"{(np.abs(got - want) / np.maximum(bound, 1e-300)).max():.2e}")
        assert excess.max() <= 0, excess.max()
        # and the rounding really happened (bfloat16 moves the product well beyond FP32 rounding)
        if precision == "bf16":
            exact = S @ x32
            assert np.abs(got - exact).max() > 1e-4 * np.abs(exact).max()


@pytest.mark.parametrize("name,mk,k,cond", CASES)
def test_bf16_mode_smoother_is_the_fp32_smoother(built, name, mk, k, cond):
    import torch
    _, P16, O = built(name, mk, k, cond, "bf16")
    _, P32, _ = built(name, mk, k, cond, "fp32")
    rng = np.random.default_rng(32)
    for l in range(len(O.S) - 1):
        r = torch.from_numpy(rng.standard_normal(O.S[l].shape[0])).cuda()
        z64 = P16.precond_apply(l, r).cpu().numpy()          # the FP64 factors
        z16 = P16.vcycle_level_apply(l, r, which=1).cpu().numpy()
        z32 = P32.vcycle_level_apply(l, r, which=1).cpu().numpy()
        e32 = np.abs(z32 - z64).max() / np.abs(z64).max()
        e16 = np.abs(z16 - z64).max() / np.abs(z64).max()
        print(f"[smoother] {name} level {l}: fp32 vs fp64 {e32:.2e}, bf16 mode vs fp64 {e16:.2e}")
        if cond == "vp":
            assert np.array_equal(z16, z32)
        assert e32 <= 1e-4 and e16 <= 3e-2


@pytest.mark.parametrize("name,mk,k,cond", CASES)
def test_bf16_fgmres_reaches_the_direct_solution(built, name, mk, k, cond):
    import oracle.solve as OS
    mesh, P, O = built(name, mk, k, cond, "bf16")
    P.set_tolerances(1e-12)                 # the error is the residual times the condition number
    x, its, hist, rel, ok = P.solve()
    P.set_tolerances(1e-10)
    assert ok and rel <= 1e-12
    xd = OS.normalise_pressure(O, OS.solve_direct(O))
    x = x.cpu().numpy()
    nf = O.lays[0].off
    ef = np.linalg.norm(x[:nf] - xd[:nf]) / np.linalg.norm(xd[:nf])
    print(f"[bf16 fgmres] {name}: its {its}, rel {rel:.2e}, face error vs direct {ef:.2e}")
    assert ef <= 1e-9
