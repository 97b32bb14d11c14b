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


PRODUCT_CASES = [CASES[0], CASES[1], CASES[2]]


@pytest.mark.parametrize("name,mk,k,cond", PRODUCT_CASES)
def test_product_copy_operator_matches_oracle_definition(name, mk, k, cond):
    """Level-0 operator of the V-cycle copy formed by the matrix-core product
    (options.vcycle_copy = PRODUCT, FP32 storage): its face blocks against the
    oracle's definition (oracle.mixed.product_copy_block: FP64 factors rounded to
    bfloat16, exact products), its couplings against the FP64 operator rounded
    to float32.  Entry by entry the difference is the FP32 accumulation of the
    cell products (at most 1e-5 of their |left||right| sums) and of the
    application (1e-5 of |S| |x|)."""
    import torch
    import scipy.sparse as sp
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    from oracle.mixed import product_copy_block
    from oracle.system import assemble_condensed
    from oracle.condense import condense_v, condense_vp
    mesh = mk()
    data = problem_data(polynomial_stokes(mesh.dim, k + 1, 3), None, mesh.dim)
    print(f"[case] product copy {name}", flush=True)
    P = H.Problem(H.Mesh(mesh), k, cond, precision="fp32", vcycle_copy="product", coarse_mode="dense",
                  rtol=1e-10)
    P.set_data(*data)
    P.bind("cuda:0")
    P.setup()
    O = OS.build(mesh, k, cond, data, eta=None)
    d, nF, nP = mesh.dim, O.lays[0].nF, O.lays[0].nP
    cfun = condense_v if cond == "v" else condense_vp
    face_blocks, bound_blocks, rest_blocks = [], [], []
    for L in O.locs:
        S, r = cfun(L)
        n = L.nfaces * d * nF
        blk, bnd = product_copy_block(L, cond)
        F = np.zeros_like(S)
        F[:n, :n] = blk
        Bd = np.zeros_like(S)
        Bd[:n, :n] = bnd
        R = S.copy()
        R[:n, :n] = 0.0
        face_blocks.append((F, r))
        bound_blocks.append((Bd, r))
        rest_blocks.append((R, r))
    Sf = assemble_condensed(mesh, face_blocks, d, nF, nP)[0]
    Sb = assemble_condensed(mesh, bound_blocks, d, nF, nP)[0]
    Sr = assemble_condensed(mesh, rest_blocks, d, nF, nP)[0]
    S_emul = (Sf + Sr).tocsr()
    S_emul.data = S_emul.data.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(41)
    x = rng.standard_normal(S_emul.shape[0])
    x32 = x.astype(np.float32).astype(np.float64)
    want = S_emul @ x32
    bound = 1e-5 * (abs(S_emul) @ np.abs(x32)) + 1e-5 * (abs(Sb) @ np.abs(x32))
    got = P.vcycle_level_apply(0, torch.from_numpy(x).cuda()).cpu().numpy()
    err = np.abs(got - want)
    print(f"[product copy] {name}: max err / bound {(err / np.maximum(bound, 1e-300)).max():.2e}")
    assert np.all(err <= bound)
    # the copy is really the product one: it differs from the FP32-rounded FP64 operator
    S32 = O.S[0].copy()
    S32.data = S32.data.astype(np.float32).astype(np.float64)
    assert np.abs(got - S32 @ x32).max() > 1e-4 * np.abs(want).max()
    # and FGMRES preconditioned by it reaches the direct solution
    P.set_tolerances(1e-12)
    xs, its, hist, rel, ok = P.solve()
    assert ok and rel <= 1e-12
    xd = OS.normalise_pressure(O, OS.solve_direct(O))
    nfv = O.lays[0].off
    assert np.linalg.norm(xs.cpu().numpy()[:nfv] - xd[:nfv]) <= 1e-9 * np.linalg.norm(xd[:nfv])


def test_product_copy_with_bf16_storage_converges():
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    mesh = cartesian_hexes(2)
    k, cond = 3, "vp"
    data = problem_data(polynomial_stokes(3, k + 1, 3), None, 3)
    print("[case] product copy, bf16 storage, hex2 k=3 vp", flush=True)
    P = H.Problem(H.Mesh(mesh), k, cond, precision="bf16", vcycle_copy="product", coarse_mode="dense", rtol=1e-12)
    P.set_data(*data)
    P.bind("cuda:0")
    P.setup()
    xs, its, hist, rel, ok = P.solve()
    assert ok and rel <= 1e-12
    O = OS.build(mesh, k, cond, data, eta=None)
    xd = OS.normalise_pressure(O, OS.solve_direct(O))
    nfv = O.lays[0].off
    assert np.linalg.norm(xs.cpu().numpy()[:nfv] - xd[:nfv]) <= 1e-9 * np.linalg.norm(xd[:nfv])
