"""GPU parity tests: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.  Tolerances are relative to the largest entry of the
compared quantity; all FP64 kernels are held to <= 1e-11 except the full V-cycle
(1e-10, nested minimal-residual steps amplify rounding).  Iterative solves are
compared iteration by iteration (FGMRES residual histories, 1e-8 per entry),
through their final iterates (library and oracle FGMRES both run to a 1e-12
relative residual agree to 1e-10) and against the exact discrete solution."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from synth import cartesian_quads, voronoi_lloyd, cartesian_hexes, polynomial_stokes, trig_series  # noqa: E402
from synth.fields import problem_data  # noqa: E402


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = [
    ("quad4_k2_v", lambda: cartesian_quads(4), 2, "v"),
    ("quad4_k2_vp", lambda: cartesian_quads(4), 2, "vp"),
    ("vor40_k3_v", lambda: voronoi_lloyd(40, 3), 3, "v"),
    ("vor40_k3_vp", lambda: voronoi_lloyd(40, 3), 3, "vp"),
    ("vor24_k1_v_neumann", lambda: voronoi_lloyd(24, 5).with_bc(lambda x: 2 if x[0] > 1 - 1e-12 else 1), 1, "v"),
    ("hex2_k2_v", lambda: cartesian_hexes(2), 2, "v"),
    ("hex2_k1_vp", lambda: cartesian_hexes(2), 1, "vp"),
]


# 3D at the highest degree the fixed-size kernels cover (face blocks of 30 rows for
# v&p-cond, the widest patch inverses)
CASES_3D_K3 = [
    ("hex2_k3_vp", lambda: cartesian_hexes(2), 3, "vp"),
    ("hex2_k3_v", lambda: cartesian_hexes(2), 3, "v"),
]


@pytest.fixture(scope="module")
def built():
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    cache = {}

    def get(name, mk, k, cond, **opts):
        key = (name, tuple(sorted(opts.items())))
        if key not in cache:
            mesh = mk()
            # polynomial data (u in P^{k+2}, p in P^{k+1}): every quadrature in both
            # implementations is exact, so the comparison is at rounding level
            data = problem_data(polynomial_stokes(mesh.dim, k + 1, 3), None, mesh.dim)
            print(f"[case] {name} k={k} cond={cond} opts={opts}", flush=True)
            M = H.Mesh(mesh)
            P = H.Problem(M, k, cond, **opts)
            P.set_data(*data)
            P.bind("cuda:0")
            P.setup()
            O = OS.build(mesh, k, cond, data, eta=None)
            cache[key] = (mesh, M, P, O)
        return cache[key]
    return get


@pytest.mark.parametrize("name,mk,k,cond", CASES)
def test_condensed_cells_and_rhs(built, name, mk, k, cond):
    import torch
    mesh, M, P, O = built(name, mk, k, cond)
    worst = 0.0
    for c in range(mesh.n_cells):
        S, r = P.condensed_cell(c)
        So, ro = O.blocks[c]
        worst = max(worst, _rel(S, So))
        assert np.abs(r - ro).max() < 1e-11 * np.abs(O.b).max()
    assert worst < 1e-11, worst
    b = P.rhs().cpu().numpy()
    assert _rel(b, O.b) < 1e-12
    torch.cuda.synchronize()


@pytest.mark.parametrize("name,mk,k,cond", CASES + CASES_3D_K3)
def test_level_operators(built, name, mk, k, cond):
    import torch
    mesh, M, P, O = built(name, mk, k, cond)
    rng = np.random.default_rng(0)
    for l, S in enumerate(O.S):
        x = rng.standard_normal(S.shape[0])
        y = P.level_apply(l, torch.from_numpy(x).cuda()).cpu().numpy()
        assert _rel(y, S @ x) < 1e-12, (l, _rel(y, S @ x))


@pytest.mark.parametrize("name,mk,k,cond", CASES + CASES_3D_K3)
def test_smoother_preconditioner(built, name, mk, k, cond):
    import torch
    import oracle.multilevel as ML
    mesh, M, P, O = built(name, mk, k, cond, coarse_mode="gmres")
    rng = np.random.default_rng(1)
    for l, S in enumerate(O.S):
        prec = ML.Schwarz(S, mesh, O.lays[l])
        r = rng.standard_normal(S.shape[0])
        z = P.precond_apply(l, torch.from_numpy(r).cuda()).cpu().numpy()
        assert _rel(z, prec(r)) < 1e-10, (l, _rel(z, prec(r)))


@pytest.mark.parametrize("name,mk,k,cond", CASES + CASES_3D_K3)
def test_vcycle_matches_oracle(built, name, mk, k, cond):
    import torch
    import oracle.solve as OS
    mesh, M, P, O = built(name, mk, k, cond, coarse_mode="dense")
    H = OS.hierarchy(O, coarse="direct")
    rng = np.random.default_rng(2)
    b = rng.standard_normal(O.S[0].shape[0])
    if O.z[0] is not None:
        b = OS.project_out(O.z[0])(b)
    x = P.vcycle_apply(torch.from_numpy(b).cuda()).cpu().numpy()
    xo = H.vcycle(0, b)
    if O.z[0] is not None:   # the coarse correction is defined up to the constant pressure
        x, xo = OS.project_out(O.z[0])(x), OS.project_out(O.z[0])(xo)
    print(f"[vcycle] {name}: {_rel(x, xo):.2e}")
    assert _rel(x, xo) < 1e-10, _rel(x, xo)


MIXED_CASES = [CASES[0], CASES[3], CASES[5], CASES_3D_K3[0]]


@pytest.mark.parametrize("name,mk,k,cond", MIXED_CASES)
def test_mixed_precision_vcycle(built, name, mk, k, cond):
    """FP32 V-cycle (levels above the coarsest in FP32, coarsest in FP64) against
    the oracle's float32 emulation of the same V-cycle (oracle.mixed: FP64
    operators and patch inverses rounded to float32, float32 vector arithmetic,
    FP64 coarsest solve) at 1e-5 of the largest entry, and against the FP64
    oracle V-cycle: it must differ from it by more than 1e-9 (FP32 is really
    used).  Each FP32 quantity carries a relative rounding of 2^-24 = 6e-8; a
    V-cycle composes some tens of them with local condition numbers below 1e2,
    so both FP32 results lie within ~1e-6 of the FP64 one."""
    import torch
    import oracle.solve as OS
    from oracle.mixed import Vcycle32
    mesh, M, P, O = built(name, mk, k, cond, coarse_mode="dense", precision="fp32")
    H = OS.hierarchy(O, coarse="direct")
    rng = np.random.default_rng(8)
    b = rng.standard_normal(O.S[0].shape[0])
    if O.z[0] is not None:
        b = OS.project_out(O.z[0])(b)
    x = P.vcycle_apply(torch.from_numpy(b).cuda()).cpu().numpy()
    xo = H.vcycle(0, b)
    x32 = Vcycle32(H)(b)
    if O.z[0] is not None:
        x, xo, x32 = (OS.project_out(O.z[0])(v) for v in (x, xo, x32))
    err64, err32 = _rel(x, xo), _rel(x, x32)
    print(f"[mixed vcycle] {name}: vs fp64 {err64:.2e}, vs fp32 emulation {err32:.2e}")
    assert err64 > 1e-9, err64          # FP32 arithmetic is really used
    assert err32 < 1e-5, err32


@pytest.mark.parametrize("name,mk,k,cond", MIXED_CASES)
def test_mixed_precision_fgmres_solution(built, name, mk, k, cond):
    """FGMRES in FP64 preconditioned by the FP32 V-cycle reaches the FP64 direct
    solution (the flexible outer iteration absorbs the FP32 preconditioner)."""
    import oracle.solve as OS
    mesh, M, P, O = built(name, mk, k, cond, coarse_mode="dense", precision="fp32", rtol=1e-11)
    x, its, hist, rel, ok = P.solve()
    assert ok and rel <= 1e-11
    xd = OS.normalise_pressure(O, OS.solve_direct(O))
    assert np.linalg.norm(x.cpu().numpy() - xd) <= 1e-8 * np.linalg.norm(xd)
    assert its <= 40


AMG_CASES = [
    ("vor120_k2_v", lambda: voronoi_lloyd(120, 7), 2, "v"),
    ("vor120_k2_vp", lambda: voronoi_lloyd(120, 7), 2, "vp"),
    ("hex4_k1_v", lambda: cartesian_hexes(4), 1, "v"),
    # 3D: coarsening stops before a nearly dense level; the coarsest AMG level
    # (1008 unknowns) gets Jacobi sweeps instead of a dense inverse
    ("hex12_k0_v", lambda: cartesian_hexes(12), 0, "v"),
]


@pytest.mark.parametrize("psmooth", [1, 2])
@pytest.mark.parametrize("explicit", [2048, 0])
@pytest.mark.parametrize("name,mk,k,cond", AMG_CASES)
def test_coarse_block_preconditioner(built, name, mk, k, cond, explicit, psmooth):
    """Coarsest-level block-triangular preconditioner with the smoothed-aggregation
    velocity block (one damped-Jacobi sweep before and after each coarse
    correction, the library's default): GPU vs the oracle's plain definition,
    with the small AMG levels applied as their explicit V-cycle matrix (2048)
    and level by level (0), with two prolongator smoothing steps (where the
    density bound allows) and one."""
    import torch
    from oracle.amg import BlockStokesPrec
    mesh, M, P, O = built(name, mk, k, cond, coarse_mode="amg", coarse_amg_explicit=explicit,
                          coarse_amg_psmooth=psmooth)
    L = len(O.S) - 1
    prec = BlockStokesPrec(O.S[L], O.lays[L].off, mesh.dim, nu=1, p_steps=psmooth)
    assert len(prec.amg.sizes) >= 2
    rng = np.random.default_rng(3)
    v = rng.standard_normal(O.S[L].shape[0])
    z = P.coarse_prec_apply(torch.from_numpy(v).cuda()).cpu().numpy()
    assert _rel(z, prec(v)) < 1e-10, _rel(z, prec(v))


def test_coarse_block_preconditioner_explicit_several_levels():
    """The explicit V-cycle matrix spanning several AMG levels, larger than one
    launch's thread count (k = 0 on 4096 Voronoi cells: the first level with at
    most 4096 rows is level 1, with levels below it): GPU vs the oracle."""
    import torch
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    from oracle.amg import BlockStokesPrec
    mesh = voronoi_lloyd(4096, 11)
    data = problem_data(polynomial_stokes(2, 1, 3), None, 2)
    P = H.Problem(H.Mesh(mesh), 0, "v", coarse_mode="amg", coarse_amg_explicit=4096)
    P.set_data(*data)
    P.bind("cuda:0", fill=0xFF)      # NaN bytes: a read of unwritten workspace shows up
    P.setup()
    O = OS.build(mesh, 0, "v", data, eta=None)
    prec = BlockStokesPrec(O.S[0], O.lays[0].off, 2, nu=1)
    sizes = prec.amg.sizes
    assert sizes[0] > 4096 and sizes[1] <= 4096 and sizes[1] ** 2 > 8192 * 256 and len(sizes) >= 4, sizes
    rng = np.random.default_rng(6)
    v = rng.standard_normal(O.S[0].shape[0])
    z = P.coarse_prec_apply(torch.from_numpy(v).cuda()).cpu().numpy()
    assert np.isfinite(z).all()
    assert _rel(z, prec(v)) < 1e-10, _rel(z, prec(v))


def test_coarse_preconditioner_independent_of_workspace_contents():
    """Property at full size (3D, 32^3 hexahedra, k = 0: 101,376 faces, B = A P
    with more entries than one launch has threads): the coarse preconditioner
    reads only what the setup wrote, so a workspace prefilled with NaN bytes and
    one prefilled with zeros give the same, finite result, bit for bit."""
    import torch
    import paper_2009_13840_amd as H
    mesh = cartesian_hexes(32)
    data = problem_data(polynomial_stokes(3, 1, 3), None, 3)
    out = []
    for fill in (0x00, 0xFF):
        P = H.Problem(H.Mesh(mesh), 0, "v", coarse_mode="amg")
        P.set_data(*data)
        P.bind("cuda:0", fill=fill)
        P.setup()
        v = torch.from_numpy(np.random.default_rng(7).standard_normal(P.level_size(0))).cuda()
        out.append(P.coarse_prec_apply(v).cpu().numpy())
        del P
    assert np.isfinite(out[0]).all() and np.isfinite(out[1]).all()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("explicit", [2048, 0])
@pytest.mark.parametrize("name,mk,k,cond", [AMG_CASES[0], AMG_CASES[3]])
def test_coarse_block_preconditioner_two_sweeps(built, name, mk, k, cond, explicit):
    """The same with two damped-Jacobi sweeps before and after each coarse correction."""
    import torch
    from oracle.amg import BlockStokesPrec
    mesh, M, P, O = built(name, mk, k, cond, coarse_mode="amg", coarse_amg_sweeps=2, coarse_amg_explicit=explicit)
    L = len(O.S) - 1
    prec = BlockStokesPrec(O.S[L], O.lays[L].off, mesh.dim, nu=2)
    rng = np.random.default_rng(4)
    v = rng.standard_normal(O.S[L].shape[0])
    z = P.coarse_prec_apply(torch.from_numpy(v).cuda()).cpu().numpy()
    assert _rel(z, prec(v)) < 1e-10, _rel(z, prec(v))


def _solution_parity(O, P, coarse, tag, **hk):
    """Library and oracle FGMRES, both to a 1e-12 relative residual with the same
    coarse solver: final iterates agree to 1e-10; both reach the direct solution."""
    import oracle.solve as OS
    x, its, hist, rel, ok = P.solve()
    assert ok and rel <= 1e-12, (its, rel)
    x = x.cpu().numpy()
    if coarse != "direct":   # the library's default coarse tolerance: 1e-3 in 3D, 1e-2 in 2D
        hk.setdefault("coarse_rtol", 1e-3 if O.mesh.dim == 3 else 1e-2)
    xo, its_o, hist_o, conv = OS.solve_fgmres(O, rtol=1e-12, coarse=coarse, **hk)
    assert conv
    xd = OS.normalise_pressure(O, OS.solve_direct(O))
    e_o = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    e_d = np.linalg.norm(x - xd) / np.linalg.norm(xd)
    print(f"[fgmres] {tag}: its {its} (oracle {its_o}), |x - x_oracle| {e_o:.2e}, |x - x_direct| {e_d:.2e}")
    assert e_o <= 1e-10, e_o
    assert e_d <= 1e-8, e_d
    assert its <= 40 and hist[0] == 1.0
    return its, its_o


@pytest.mark.parametrize("name,mk,k,cond", AMG_CASES)
def test_fgmres_solution_amg_coarse(built, name, mk, k, cond):
    mesh, M, P, O = built(name, mk, k, cond, coarse_mode="amg", rtol=1e-12)
    _solution_parity(O, P, "amg", name)


@pytest.mark.parametrize("name,mk,k,cond", [AMG_CASES[0]])
def test_fgmres_solution_long_coarse_cycles(built, name, mk, k, cond):
    """Coarse GMRES with 64-vector cycles run to a tight tolerance, so a cycle
    reaches the columns past the fused one-pass Gram-Schmidt's 64 sums."""
    import oracle.solve as OS
    mesh, M, P, O = built(name, mk, k, cond, coarse_mode="gmres", coarse_restart=64, coarse_rtol=1e-14,
                          coarse_max_it=70, rtol=1e-11)
    x, its, hist, rel, ok = P.solve()
    assert ok and rel <= 1e-11
    tm = P.timings()
    assert tm["coarse_its"] > 63 * tm["vcycles"], tm     # every coarse solve ran past column 63
    xd = OS.normalise_pressure(O, OS.solve_direct(O))
    assert np.linalg.norm(x.cpu().numpy() - xd) <= 1e-8 * np.linalg.norm(xd)


@pytest.mark.parametrize("name,mk,k,cond", CASES)
@pytest.mark.parametrize("coarse", ["dense", "gmres", "direct"])
def test_fgmres_solution(built, name, mk, k, cond, coarse):
    mesh, M, P, O = built(name, mk, k, cond, coarse_mode=coarse, rtol=1e-12)
    exact = coarse in ("dense", "direct")     # both solve the coarsest level exactly
    its, its_o = _solution_parity(O, P, "direct" if exact else "gmres", f"{name} {coarse}")
    if exact:
        assert its == its_o


@pytest.mark.parametrize("coarse", ["dense", "direct"])
@pytest.mark.parametrize("restart", [30, 3])
@pytest.mark.parametrize("name,mk,k,cond", CASES + CASES_3D_K3)
def test_fgmres_history_matches_oracle(built, name, mk, k, cond, restart, coarse):
    """Iteration-level parity of flexible GMRES (CGS2 Arnoldi, Givens rotations,
    restarts from the true residual): with the exact coarsest solve (bordered
    dense inverse, or the sparse direct solver) the V-cycle is the same linear
    map on both sides, so the library and the oracle take the same number of
    iterations and their relative residual estimates agree to 1e-8 per entry
    while above 1e-8.  Restart 3 forces several restarts."""
    import oracle.solve as OS
    mesh, M, P, O = built(name, mk, k, cond, coarse_mode=coarse, rtol=1e-10, restart=restart)
    x, its, hist, rel, ok = P.solve()
    assert ok
    xo, its_o, hist_o, conv = OS.solve_fgmres(O, rtol=1e-10, restart=restart, coarse="direct")
    ho = np.asarray(hist_o)
    print(f"[history] {name} {coarse} restart {restart}: its {its} (oracle {its_o})")
    assert its == its_o and len(hist) == len(ho)
    sel = ho > 1e-8
    assert sel.sum() >= 3
    dev = np.abs(hist[sel] - ho[sel]) / ho[sel]
    print(f"[history] {name} {coarse} restart {restart}: max per-entry deviation {dev.max():.2e}")
    assert dev.max() <= 1e-8, dev.max()


@pytest.mark.parametrize("name,mk,k,cond", CASES + CASES_3D_K3 + [
    ("quad4_k0_v", lambda: cartesian_quads(4), 0, "v"),
    ("hex1_k0_vp", lambda: cartesian_hexes(1), 0, "vp"),      # one pressure mode: nothing to eliminate
])
def test_recover_cells(built, name, mk, k, cond):
    """Cell unknowns eliminated by static condensation, recovered on the device
    from a random vector and from the FGMRES solution, against the oracle's dense
    local solves (v&p-cond also recovers the non-mean pressure modes)."""
    import torch
    import oracle.solve as OS
    mesh, M, P, O = built(name, mk, k, cond, rtol=1e-11)
    rng = np.random.default_rng(21)
    xs = [rng.standard_normal(P.level_size(0))]
    x, its, hist, rel, ok = P.solve()
    assert ok
    xs.append(x.cpu().numpy())
    for x in xs:
        u, p = P.recover_cells(torch.from_numpy(x).cuda())
        uo, po = OS.recover(O, x)
        assert u.shape == uo.shape and p.shape == po.shape
        assert _rel(u.cpu().numpy(), uo) < 1e-11, _rel(u.cpu().numpy(), uo)
        assert _rel(p.cpu().numpy(), po) < 1e-11, _rel(p.cpu().numpy(), po)


DEGENERATE_CASES = [
    ("quad1_k0_v", lambda: cartesian_quads(1), 0, "v"),       # one cell, one level (bordered dense solve)
    ("hex1_k0_vp", lambda: cartesian_hexes(1), 0, "vp"),
    ("quad4_k0_v", lambda: cartesian_quads(4), 0, "v"),       # one level: the V-cycle is the coarse solve
    ("quad2_k2_vp", lambda: cartesian_quads(2), 2, "vp"),     # the smallest multilevel case (4 cells)
    ("hex2_k1_v_two_levels", lambda: cartesian_hexes(2), 1, "v"),
]


@pytest.mark.parametrize("name,mk,k,cond", DEGENERATE_CASES)
def test_degenerate_problems(built, name, mk, k, cond):
    """Single-cell meshes, a single-level hierarchy and the smallest multilevel
    meshes: level operators, and FGMRES reaching the direct solution."""
    import torch
    import oracle.solve as OS
    mesh, M, P, O = built(name, mk, k, cond, rtol=1e-11)
    rng = np.random.default_rng(9)
    for l, S in enumerate(O.S):
        x = rng.standard_normal(S.shape[0])
        y = P.level_apply(l, torch.from_numpy(x).cuda()).cpu().numpy()
        assert _rel(y, S @ x) < 1e-12, (l, _rel(y, S @ x))
    x, its, hist, rel, ok = P.solve()
    assert ok and rel <= 1e-11
    xd = OS.normalise_pressure(O, OS.solve_direct(O))
    assert np.linalg.norm(x.cpu().numpy() - xd) <= 1e-8 * np.linalg.norm(xd)


def test_single_cell_patch_holding_the_pressure_null_space_is_reported():
    """With one cell and k >= 1 the only smoother patch holds the constant
    pressure, the null space of the all-Dirichlet problem, so it is singular:
    setup fails with HHO_E_LOCAL_SINGULAR instead of producing a garbage smoother."""
    import paper_2009_13840_amd as H
    mesh = cartesian_quads(1)
    data = problem_data(polynomial_stokes(2, 2, 3), None, 2)
    P = H.Problem(H.Mesh(mesh), 1, "v")
    P.set_data(*data)
    P.bind("cuda:0")
    with pytest.raises(H.HHOError) as e:
        P.setup()
    assert "not invertible" in str(e.value)


def test_autotune_keeps_solution(built):
    """The autotuner only changes launch shapes: the solve still reaches the direct solution."""
    import oracle.solve as OS
    name, mk, k, cond = CASES[2]
    mesh, M, P, O = built(name, mk, k, cond, coarse_mode="dense", rtol=1e-11)
    ch = P.autotune(reps=3)
    assert ch.shape == (len(O.S), 2)
    assert set(ch[:, 0]) <= {64, 128, 256} and set(ch[:-1, 1]) <= {0, 64, 128, 256, 512}
    x, its, hist, rel, ok = P.solve()
    xd = OS.normalise_pressure(O, OS.solve_direct(O))
    assert ok and np.linalg.norm(x.cpu().numpy() - xd) <= 1e-8 * np.linalg.norm(xd)
