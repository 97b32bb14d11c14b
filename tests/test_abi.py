"""CPU tests of the C ABI: the library loads and exports every declared symbol,
argument validation and error codes, and the host-built local HHO operators
against the oracle (no device calls)."""
import os
import re

import numpy as np
import pytest

from synth import cartesian_quads, voronoi_lloyd, cartesian_hexes, polynomial_stokes
from synth.fields import problem_data

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2009_13840_amd as H
    return H, H.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hho_pmg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hho_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    H, lib = _lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(H.EXPORTS)


def test_mesh_validation_errors():
    H, _ = _lib()
    m = cartesian_quads(2)
    bad = cartesian_quads(2)
    bad.face_bc = bad.face_bc.copy()
    bad.face_bc[np.argmax(bad.face_bc)] = 0      # boundary face without a boundary flag
    with pytest.raises(H.HHOError) as e:
        H.Mesh(bad)
    assert e.value.code == -2
    bad2 = cartesian_quads(2)
    bad2.face_bc = bad2.face_bc.copy()
    bad2.face_bc[np.argmin(bad2.face_bc)] = 1    # interior face with a boundary flag
    with pytest.raises(H.HHOError) as e:
        H.Mesh(bad2)
    assert e.value.code == -2
    H.Mesh(m)


def test_problem_argument_validation():
    H, _ = _lib()
    M = H.Mesh(cartesian_quads(2))
    for kw in (dict(k=-1), dict(k=7), dict(k=2, degrees=[2, 2, 0]), dict(k=2, degrees=[1, 0]),
               dict(k=1, restart=0), dict(k=1, smooth_its=3), dict(k=1, coarse_amg_sweeps=3),
               dict(k=1, coarse_amg_explicit=-1), dict(k=1, coarse_amg_explicit=4097),
               dict(k=1, coarse_amg_psmooth=0), dict(k=1, coarse_amg_psmooth=3)):
        k = kw.pop("k")
        with pytest.raises(H.HHOError) as e:
            H.Problem(M, k, "v", **kw)
        assert e.value.code == -1, kw
    P = H.Problem(M, 1, "v")
    with pytest.raises(H.HHOError) as e:
        P.workspace_size()                        # before set_data
    assert e.value.code == -1
    with pytest.raises(H.HHOError) as e:
        P.setup()
    assert e.value.code == -1


def test_recover_cells_requires_setup_and_buffers():
    """Host-side checks of hho_recover_cells, taken before any device work."""
    import ctypes as C
    H, lib = _lib()
    P = H.Problem(H.Mesh(cartesian_quads(2)), 1, "v")
    P.set_data(*problem_data(polynomial_stokes(2, 1, 0), None, 2))
    dummy = C.c_void_p(0x1000)
    assert lib.hho_recover_cells(P.h, dummy, dummy, dummy) == -1      # no setup yet
    assert b"hho_setup" in lib.hho_last_error()
    assert lib.hho_recover_cells(None, dummy, dummy, dummy) == -1


def test_workspace_capacity_error():
    import ctypes as C
    H, lib = _lib()
    P = H.Problem(H.Mesh(cartesian_quads(2)), 1, "v")
    P.set_data(*problem_data(polynomial_stokes(2, 1, 0), None, 2))
    n = P.workspace_size()
    assert n > 0
    code = lib.hho_bind_workspace(P.h, C.c_void_p(0x1000), n - 1)
    assert code == -7


@pytest.mark.parametrize("mesh,k", [(cartesian_quads(3), 1), (voronoi_lloyd(20, 3), 3), (cartesian_hexes(2), 2),
                                    (cartesian_quads(3).with_bc(lambda x: 2 if x[0] > 1 - 1e-12 else 1), 2)])
def test_host_local_operators_match_oracle(mesh, k):
    """The library's host-built local operators (its own quadrature, bases and
    integrated-by-parts coupling) equal the oracle's to rounding."""
    H, _ = _lib()
    from oracle.hho import mesh_geometry, local_hho
    from oracle.solve import default_eta
    data = problem_data(polynomial_stokes(mesh.dim, k, 5), None, mesh.dim)
    P = H.Problem(H.Mesh(mesh), k, "v")
    P.set_data(*data)
    geo = mesh_geometry(mesh, k)
    for c in range(mesh.n_cells):
        L = local_hho(mesh, geo, c, default_eta(mesh, k), *data)
        G = P.local_cell(c)
        assert np.abs(G["a"] - L.a).max() <= 1e-12 * np.abs(L.a).max()
        assert np.abs(G["B"] - L.B).max() <= 1e-12 * np.abs(L.B).max()
        assert np.abs(G["rhs_u"] - L.rhs_u).max() <= 1e-12 * max(1.0, np.abs(L.rhs_u).max())
        assert np.abs(G["rhs_p"] - L.rhs_p).max() <= 1e-12 * max(1.0, np.abs(L.rhs_p).max())


def test_union_mesh_and_segment_validation():
    H, _ = _lib()
    a, b = cartesian_quads(2), voronoi_lloyd(10, 1)
    U, fo, co = H.Mesh.union([a, b])
    assert list(fo) == [0, a.n_faces, a.n_faces + b.n_faces]
    assert list(co) == [0, a.n_cells, a.n_cells + b.n_cells]
    assert (U.n_faces, U.n_cells) == (fo[-1], co[-1])
    P = H.Problem(U, 1, "v", coarse_mode="amg")
    with pytest.raises(H.HHOError) as e:            # ranges that do not partition the faces
        P.set_segments([0, 3, fo[-1] - 1], co)
    assert e.value.code == -1
    with pytest.raises(H.HHOError) as e:            # a cell whose faces lie in another member
        P.set_segments([0, fo[1] + 1, fo[2]], co)
    assert e.value.code == -1
    P.set_segments(fo, co)
    with pytest.raises(H.HHOError) as e:            # dense coarse solver with per-member null spaces
        Q = H.Problem(U, 1, "v", coarse_mode="dense")
        Q.set_segments(fo, co)
    assert e.value.code == -1


def test_batch_refuses_mixed_boundary_types():
    """A batch is a set of independent problems: a member with Neumann faces beside
    one without would need a pressure null space for some members only."""
    H, _ = _lib()
    from synth.batch import shifted
    a = cartesian_quads(3)
    b = shifted(cartesian_quads(3), 2.0).with_bc(lambda x: 2 if x[0] > 3 - 1e-12 else 1)
    U, fo, co = H.Mesh.union([a, b])
    P = H.Problem(U, 1, "v")
    with pytest.raises(H.HHOError, match="Neumann"):
        P.set_segments(fo, co)


def test_batch_members_take_their_own_penalty():
    """The default Nitsche penalty depends on max card(F_T); in a batch each member
    takes its own (a quadrilateral member beside a Voronoi member keeps the
    quadrilateral's penalty), so its local operators are those it has alone."""
    H, _ = _lib()
    from synth.batch import shifted, region_fields
    quads, vor = cartesian_quads(3), voronoi_lloyd(20, 4)
    fields = [problem_data(polynomial_stokes(2, 2, 5 + i), None, 2) for i in range(2)]
    U, fo, co = H.Mesh.union([quads, shifted(vor, 2.0)])
    P = H.Problem(U, 1, "v")
    P.set_segments(fo, co)
    P.set_data(*region_fields(fields, 2, 2.0))
    A = H.Problem(H.Mesh(quads), 1, "v")
    A.set_data(*fields[0])
    for c in range(quads.n_cells):
        u, a = P.local_cell(c), A.local_cell(c)
        assert np.abs(u["a"] - a["a"]).max() <= 1e-12 * np.abs(a["a"]).max()
