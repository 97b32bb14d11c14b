"""The seeded input generators (no method arithmetic): reproducible for a seed,
different across seeds, and producing valid inputs (closed meshes that tile the
unit box, bounded batch specifications)."""
import numpy as np

from synth import voronoi_lloyd, cartesian_hexes, cartesian_quads, trig_series
from synth.batch import batch_spec


def _tiles_unit_box(mesh):
    from oracle.geometry import cell_geometry, face_geometry
    fg = [face_geometry(mesh, f) for f in range(mesh.n_faces)]
    vol = sum(cell_geometry(mesh, c, fg).volume for c in range(mesh.n_cells))
    fc = mesh.face_cells()
    interior = fc[:, 1] >= 0
    return abs(vol - 1.0) < 1e-12 and np.array_equal(mesh.face_bc != 0, ~interior)


def test_voronoi_reproducible_and_valid():
    a, b, c = voronoi_lloyd(64, 3), voronoi_lloyd(64, 3), voronoi_lloyd(64, 4)
    assert a.n_cells == 64
    assert np.array_equal(a.verts, b.verts) and np.array_equal(a.cell_face, b.cell_face)
    assert a.verts.shape != c.verts.shape or not np.allclose(a.verts, c.verts)
    assert _tiles_unit_box(a)


def test_cartesian_meshes_valid():
    h = cartesian_hexes(2)
    assert (h.n_cells, h.n_faces, int((h.face_bc != 0).sum())) == (8, 36, 24)
    assert _tiles_unit_box(h) and _tiles_unit_box(cartesian_quads(3))


def test_trig_series_reproducible():
    x = np.random.default_rng(0).random((50, 2))
    f1, f2, g = trig_series(2, 7), trig_series(2, 7), trig_series(2, 8)
    assert np.array_equal(f1(x), f2(x))
    assert not np.allclose(f1(x), g(x))


def test_batch_spec_reproducible_and_bounded():
    s1, s2 = batch_spec(), batch_spec()
    assert s1 == s2 and len(s1) == 256
    sides = np.array([s for s, _, _ in s1])
    ks = np.array([k for _, k, _ in s1])
    assert sides.min() >= 16 and sides.max() <= 96 and ks.min() >= 1 and ks.max() <= 4
    assert len({seed for _, _, seed in s1}) == 256


def test_trig_series_matches_its_definition():
    """The contracted evaluation equals the sum over alpha written out, in 2D and 3D,
    on enough points to take the threaded blocks."""
    rng = np.random.default_rng(5)
    for dim in (2, 3):
        T = trig_series(dim, 11)
        x = rng.random((300_000, dim))
        y = T(x)
        idx = rng.integers(0, x.shape[0], 64)
        xs = x[idx]
        ref = np.zeros((64, dim))
        for i, al in enumerate(T.alphas):
            ref += np.outer(np.prod(np.cos(np.pi * al * xs), axis=1), T.a[:, i])
            ref += np.outer(np.prod(np.sin(np.pi * al * xs), axis=1), T.b[:, i])
        assert np.abs(y[idx] - ref).max() <= 1e-12 * np.abs(ref).max()
