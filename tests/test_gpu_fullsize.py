"""Parity at the full size of the workloads the benchmark times: the 2D Voronoi
problem (16384 Lloyd-relaxed cells, seed 2, k = 3, levels 3-2-1-0, v-cond and
v&p-cond, default options) and the 3D ones (32^3 hexahedra, k = 3, v&p-cond, FP32
V-cycle under FP64 FGMRES; 32^3 hexahedra, k = 2, v&p-cond; 24^3 hexahedra,
k = 3, v-cond), with polynomial data so that both sides integrate exactly.

The oracle cannot assemble the whole system in seconds, so it builds the local
operators only for the cells around a seeded sample (two rings of neighbours)
and checks the library's outputs at the sample's rows, one row at a time:
condensed cell blocks and right-hand side (eqs. ST.1 / ST.2), the fine operator
(face rows are sums over the face's two cells, pressure rows belong to one
cell) and every coarse operator at the sample's rows, the cell-patch Schwarz smoother (a face's correction is the weighted sum
of its two patches' solutions), and, after a full FGMRES solve, the residual
of the library's solution at the sampled face rows, formed from the oracle's own
rows of the operator and right-hand side.  A CPU test checks the sampled row
assembly against the oracle's full assembly on a small mesh."""
import numpy as np
import pytest

from synth import voronoi_lloyd, polynomial_stokes
from synth.fields import problem_data

N_CELLS, MESH_SEED, K = 16384, 2, 3


def _ring(mesh, fc, cells, depth):
    """cells plus every cell reached through at most `depth` shared faces"""
    out, front = set(cells), set(cells)
    for _ in range(depth):
        nxt = set()
        for c in front:
            for f in mesh.cell_faces(c):
                for t in fc[f]:
                    if t >= 0 and int(t) not in out:
                        nxt.add(int(t))
        out |= nxt
        front = nxt
    return sorted(out)


class SampledOracle:
    """Oracle rows of the level-0 condensed system around a set of cells."""

    def __init__(self, mesh, k, cond, data, sample):
        from oracle.bases import FaceBasis, dim_poly
        from oracle.condense import condense_v, condense_vp
        from oracle.geometry import cell_geometry, face_geometry, face_quadrature
        from oracle.hho import Geometry, local_hho
        from oracle.solve import default_eta
        from oracle.system import face_dofs, layout
        self.mesh, self.d = mesh, mesh.dim
        self.fc = mesh.face_cells()
        self.sample = sorted(int(c) for c in sample)
        self.ring1 = _ring(mesh, self.fc, self.sample, 1)
        self.ring2 = _ring(mesh, self.fc, self.sample, 2)
        qdeg = 2 * k + 8      # well above what the polynomial data needs
        nf, nc = mesh.n_faces, mesh.n_cells
        fgeo, fq, fb, cgeo = [None] * nf, [None] * nf, [None] * nf, [None] * nc
        for c in self.ring2:
            for f in mesh.cell_faces(c):
                if fgeo[f] is None:
                    fgeo[f] = face_geometry(mesh, f)
                    fq[f] = face_quadrature(mesh, fgeo[f], qdeg)
                    fb[f] = FaceBasis(fgeo[f], fq[f][0], fq[f][1], k)
            cgeo[c] = cell_geometry(mesh, c, fgeo)
        geo = Geometry(fgeo, cgeo, fq, fb, k, qdeg)
        eta = default_eta(mesh, k)
        cfun = condense_v if cond == "v" else condense_vp
        self.lay = layout(mesh, k, cond)
        self.nF, self.nP = self.lay.nF, self.lay.nP
        self.blocks, self.idx = {}, {}
        for c in self.ring2:
            self.blocks[c] = cfun(local_hho(mesh, geo, c, eta, *data))
            self.idx[c] = np.concatenate([face_dofs(mesh, c, self.d, self.nF),
                                          self.lay.off + c * self.nP + np.arange(self.nP)])
        self.N = self.lay.off + nc * self.nP
        assert dim_poly(self.d - 1, k) == self.nF

    def face_rows(self, f):
        return (f * self.d) * self.nF + np.arange(self.d * self.nF)

    def rows(self):
        """face rows of the sample's faces and pressure rows of the sample's cells"""
        faces = sorted({int(f) for c in self.sample for f in self.mesh.cell_faces(c)})
        r = [self.face_rows(f) for f in faces]
        r += [self.lay.off + c * self.nP + np.arange(self.nP) for c in self.sample]
        return np.concatenate(r), np.concatenate([self.face_rows(f) for f in faces])

    def apply(self, x, rows):
        """(S x)[rows]: every cell adjacent to a face of the sample contributes"""
        y = np.zeros(self.N)
        for c in self.ring1:
            idx = self.idx[c]
            y[idx] += self.blocks[c][0] @ x[idx]
        return y[rows]

    def rhs(self, rows):
        b = np.zeros(self.N)
        for c in self.ring1:
            b[self.idx[c]] += self.blocks[c][1]
        return b[rows]

    def _patch(self, c):
        """level-0 matrix of the patch of cell c (c in ring 1: all its entries come from ring 2)"""
        idx = self.idx[c]
        pos = {int(g): i for i, g in enumerate(idx)}
        A = np.zeros((len(idx), len(idx)))
        for t in _ring(self.mesh, self.fc, [c], 1):
            jt = self.idx[t]
            loc = [(a, pos[int(g)]) for a, g in enumerate(jt) if int(g) in pos]
            la, lp = np.array([u for u, _ in loc]), np.array([v for _, v in loc])
            A[np.ix_(lp, lp)] += self.blocks[t][0][np.ix_(la, la)]
        return A

    def schwarz(self, r, rows):
        """additive Schwarz with face weights 1 / card(T_F), at rows of the sample"""
        z = np.zeros(self.N)
        for c in self.ring1:
            idx = self.idx[c]
            nfc = len(self.mesh.cell_faces(c))
            w = np.concatenate([np.repeat(1.0 / (self.fc[self.mesh.cell_faces(c)] >= 0).sum(axis=1),
                                          self.d * self.nF), np.ones(self.nP)])
            assert len(w) == len(idx) == nfc * self.d * self.nF + self.nP
            z[idx] += w * np.linalg.solve(self._patch(c), r[idx])
        return z[rows]


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _sample(mesh, fc, rng, n):
    """n seeded cells, the first one touching the boundary"""
    bnd = [int(fc[f, 0]) for f in range(mesh.n_faces) if fc[f, 1] < 0]
    cells = {bnd[int(rng.integers(len(bnd)))]}
    while len(cells) < n:
        cells.add(int(rng.integers(mesh.n_cells)))
    return sorted(cells)


def test_sampled_oracle_rows_match_full_assembly():
    """CPU: the sampled rows (operator, right-hand side, Schwarz smoother) equal
    those of the oracle's full assembly on a small mesh."""
    import oracle.solve as OS
    import oracle.multilevel as ML
    mesh = voronoi_lloyd(60, 4)
    data = problem_data(polynomial_stokes(2, 3, 3), None, 2)
    for cond in ("v", "vp"):
        O = OS.build(mesh, 2, cond, data, eta=None)
        so = SampledOracle(mesh, 2, cond, data, _sample(mesh, mesh.face_cells(), np.random.default_rng(1), 3))
        rows, _ = so.rows()
        x = np.random.default_rng(2).standard_normal(O.S[0].shape[0])
        assert _rel(so.apply(x, rows), (O.S[0] @ x)[rows]) < 1e-12
        assert _rel(so.rhs(rows), O.b[rows]) < 1e-12
        prec = ML.Schwarz(O.S[0], mesh, O.lays[0])
        assert _rel(so.schwarz(x, rows), prec(x)[rows]) < 1e-10
        # coarse rows through the zero-padded fine vector
        from oracle.system import coarse_indices
        idx = np.arange(O.S[0].shape[0])
        for l in range(1, len(O.S)):
            idx = idx[coarse_indices(O.lays[l - 1], O.lays[l])]
            xl = np.random.default_rng(3 + l).standard_normal(len(idx))
            xf = np.zeros(O.S[0].shape[0])
            xf[idx] = xl
            sel = np.flatnonzero(np.isin(idx, rows))
            assert len(sel) > 0
            assert _rel(so.apply(xf, idx[sel]), (O.S[l] @ xl)[sel]) < 1e-12


@pytest.fixture(scope="module")
def workload():
    mesh = voronoi_lloyd(N_CELLS, MESH_SEED)
    return mesh, mesh.face_cells()


@pytest.mark.gpu
@pytest.mark.parametrize("cond", ["v", "vp"])
def test_full_size_voronoi_k3(workload, cond):
    mesh, fc = workload
    print(f"[case] voronoi{N_CELLS} k={K} cond={cond}", flush=True)
    _check_full_size(mesh, fc, cond, nsample=8, seed=5)


@pytest.mark.gpu
def test_full_size_hex32_k3_vp_fp32_vcycle():
    from synth import cartesian_hexes
    mesh = cartesian_hexes(32)
    print("[case] hex32 k=3 cond=vp precision=fp32", flush=True)
    _check_full_size(mesh, mesh.face_cells(), "vp", nsample=3, seed=6, precision="fp32")


@pytest.mark.gpu
def test_full_size_hex32_k2_vp():
    from synth import cartesian_hexes
    mesh = cartesian_hexes(32)
    print("[case] hex32 k=2 cond=vp", flush=True)
    _check_full_size(mesh, mesh.face_cells(), "vp", nsample=3, seed=7, k=2)


@pytest.mark.gpu
def test_full_size_hex24_k3_v():
    from synth import cartesian_hexes
    mesh = cartesian_hexes(24)
    print("[case] hex24 k=3 cond=v", flush=True)
    _check_full_size(mesh, mesh.face_cells(), "v", nsample=3, seed=8)


def _check_full_size(mesh, fc, cond, nsample, seed, k=K, **opts):
    import torch
    import paper_2009_13840_amd as H
    from oracle.system import layout, coarse_indices
    d = mesh.dim
    data = problem_data(polynomial_stokes(d, k + 1, 3), None, d)
    P = H.Problem(H.Mesh(mesh), k, cond, **opts)
    P.set_data(*data)
    P.bind("cuda:0")
    P.setup()
    rng = np.random.default_rng(seed)
    so = SampledOracle(mesh, k, cond, data, _sample(mesh, fc, rng, nsample))
    rows, frows = so.rows()
    N = P.level_size(0)
    assert N == so.N
    # condensed blocks of the sampled cells
    for c in so.sample:
        S, r = P.condensed_cell(c)
        So, ro = so.blocks[c]
        assert _rel(S, So) < 1e-11, (c, _rel(S, So))
        assert _rel(r, ro) < 1e-11, (c, _rel(r, ro))
    # condensed right-hand side and fine operator at the sample's rows
    b = P.rhs().cpu().numpy()
    assert _rel(b[rows], so.rhs(rows)) < 1e-11
    x = rng.standard_normal(N)
    y = P.level_apply(0, torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.isfinite(y).all()
    assert _rel(y[rows], so.apply(x, rows)) < 1e-11
    # coarse operators k-1 ... 0 (sub-blocks of the fine one, Section 4.2): at the
    # sample's rows S_l x_l equals the fine rows of S_0 (P x_l), P the zero-padding
    lays = [layout(mesh, kl, cond) for kl in range(k, -1, -1)]
    idx = np.arange(N)                       # fine index of every level-l unknown
    for l in range(1, len(lays)):
        idx = idx[coarse_indices(lays[l - 1], lays[l])]
        assert P.level_size(l) == len(idx)
        xl = rng.standard_normal(len(idx))
        yl = P.level_apply(l, torch.from_numpy(xl).cuda()).cpu().numpy()
        assert np.isfinite(yl).all()
        sel = np.flatnonzero(np.isin(idx, rows))
        assert len(sel) > 0
        xf = np.zeros(N)
        xf[idx] = xl
        assert _rel(yl[sel], so.apply(xf, idx[sel])) < 1e-11, (l, _rel(yl[sel], so.apply(xf, idx[sel])))
    # patch smoother
    z = P.precond_apply(0, torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.isfinite(z).all()
    assert _rel(z[rows], so.schwarz(x, rows)) < 1e-10
    # full solve: residual at the sampled face rows from the oracle's rows
    xs, its, hist, rel, ok = P.solve()
    assert ok and rel <= 1e-8, (its, rel)
    xs = xs.cpu().numpy()
    res = so.rhs(frows) - so.apply(xs, frows)
    assert np.abs(res).max() <= 2e-8 * np.linalg.norm(b), (np.abs(res).max(), np.linalg.norm(b))


@pytest.mark.gpu
def test_batch256_sampled_members_match_oracle():
    """The benchmark's batch at full scale: 256 problems (Cartesian sides 16..96,
    k 1..4, trig-series forcing seeds 4000+i), one disjoint-union problem per
    degree with per-member FGMRES, V-cycle coefficients and coarse GMRES, FP32
    V-cycle, solved to 1e-12.  In every degree group the two smallest members are
    compared with the oracle's direct solve of that member alone (faces to 1e-8:
    the member's local operators are formed on its shifted copy, which moves
    them at rounding level), and every member meets the tolerance."""
    import paper_2009_13840_amd as H
    import oracle.solve as OS
    from synth import cartesian_quads, trig_series
    from synth.batch import batch_spec, shifted, region_fields
    spec = batch_spec()
    groups = {}
    for i, (side, k, seed) in enumerate(spec):
        groups.setdefault(k, []).append((i, side, seed))
    width = 2.0
    for k, mem in sorted(groups.items()):
        print(f"[case] batch256 degree {k}: {len(mem)} members", flush=True)
        meshes = [cartesian_quads(side) for (_, side, _) in mem]
        fields = [problem_data(None, trig_series(2, seed), 2) for (_, _, seed) in mem]
        U, fo, co = H.Mesh.union([shifted(m, width * j) for j, m in enumerate(meshes)])
        P = H.Problem(U, k, "v", precision="fp32", rtol=1e-12)
        P.set_segments(fo, co)
        P.set_data(*region_fields(fields, 2, width))
        P.bind("cuda:0")
        P.setup()
        x, its, hist, rel, ok = P.solve()
        m_its, m_rel = P.batch_results()
        assert ok and np.all(m_rel <= 1e-12), (k, m_rel.max())
        x = x.cpu().numpy()
        nface_total = int(fo[-1])
        for j in sorted(range(len(mem)), key=lambda j: mem[j][1])[:2]:
            O = OS.build(meshes[j], k, "v", fields[j], eta=None)
            xd = OS.normalise_pressure(O, OS.solve_direct(O))
            dp = 2 * O.lays[0].nF
            xf = x[fo[j] * dp:fo[j + 1] * dp]
            err = np.linalg.norm(xf - xd[:xf.size]) / np.linalg.norm(xd[:xf.size])
            print(f"[batch256] degree {k} member {mem[j][0]} (side {mem[j][1]}): its {m_its[j]}, "
                  f"face error vs direct {err:.1e}", flush=True)
            assert err <= 1e-8, (k, j, err)
        del P
