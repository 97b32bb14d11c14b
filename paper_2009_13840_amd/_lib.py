"""ctypes binding of ``libhho_pmg.so`` (argument marshalling only).

Every computation happens in the HIP library: this module converts Python/NumPy
arguments to the C ABI of ``include/hho_pmg.h``, allocates the device
workspace as a torch uint8 tensor and passes torch's current HIP stream.  It
fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhho_pmg.so")

HHO_OK = 0
ERRORS = {-1: "HHO_E_INVALID_ARG", -2: "HHO_E_MESH", -3: "HHO_E_LOCAL_SINGULAR", -4: "HHO_E_NOT_CONVERGED",
          -5: "HHO_E_BREAKDOWN", -6: "HHO_E_DEVICE", -7: "HHO_E_CAPACITY", -8: "HHO_E_OOM"}
COND = {"v": 1, "vp": 2}
PROBE = {"operator": 1, "smoother": 2, "coarse_operator": 4, "outer_operator": 8, "amg_restrict": 16,
         "amg_sweep": 32, "amg_prolong": 64, "amg_dense": 128, "direct_fwd": 256, "direct_bwd": 512}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
COARSE = {"auto": 0, "dense": 1, "gmres": 2, "amg": 3, "direct": 4}
COPY = {"convert": 0, "product": 1}
LOCAL = {"auto": 0, "host": 1, "device": 2}
SMOOTHER = {"schwarz": 0, "ilu": 1}

EXPORTS = ["hho_last_error", "hho_options_default", "hho_mesh_create", "hho_mesh_destroy", "hho_problem_create",
           "hho_problem_destroy", "hho_problem_set_data", "hho_workspace_size", "hho_bind_workspace",
           "hho_set_stream", "hho_set_graph", "hho_setup", "hho_level_size", "hho_solve", "hho_solve_device", "hho_solution_sizes",
           "hho_moments_size", "hho_set_moments", "hho_batch_create", "hho_batch_destroy", "hho_batch_problem",
           "hho_batch_sizes", "hho_batch_solve", "hho_learned_save", "hho_learned_load", "hho_get_rhs", "hho_get_condensed_cell",
           "hho_get_local_cell", "hho_local_hp_cell", "hho_hp_skeleton", "hho_level_apply", "hho_vcycle_level_apply", "hho_precond_apply", "hho_vcycle_apply", "hho_get_timings", "hho_upload",
           "hho_time_kernel", "hho_coarse_prec_apply", "hho_coarse_solve_apply", "hho_direct_info", "hho_debug_copy", "hho_learned_dims",
           "hho_learned_set_params", "hho_learned_get_params", "hho_learned_enable", "hho_learned_apply",
           "hho_learned_collect", "hho_learned_grad", "hho_learned_grad_noalloc", "hho_learned_train", "hho_mesh_create_union",
           "hho_problem_set_segments", "hho_batch_results", "hho_autotune", "hho_recover_cells",
           "hho_set_tolerances", "hho_probe_arm", "hho_probe_read", "hho_probe_clear", "hho_amg_level_info"]


class HHOError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_verts", C.c_int64), ("verts", C.POINTER(C.c_double)),
                ("n_faces", C.c_int64), ("face_ptr", C.POINTER(C.c_int64)), ("face_vtx", C.POINTER(C.c_int64)),
                ("n_cells", C.c_int64), ("cell_ptr", C.POINTER(C.c_int64)), ("cell_face", C.POINTER(C.c_int64)),
                ("face_bc", C.POINTER(C.c_int8))]


class Options(C.Structure):
    _fields_ = [("eta", C.c_double), ("rtol", C.c_double), ("max_it", C.c_int32), ("restart", C.c_int32),
                ("smooth_its", C.c_int32), ("precision", C.c_int32), ("coarse_mode", C.c_int32),
                ("coarse_rtol", C.c_double), ("coarse_restart", C.c_int32), ("coarse_max_it", C.c_int32),
                ("quad_extra", C.c_int32), ("coarse_amg_sweeps", C.c_int32), ("learned", C.c_int32),
                ("coarse_amg_explicit", C.c_int32), ("coarse_amg_psmooth", C.c_int32), ("smoother", C.c_int32),
                ("nullspace", C.c_int32), ("vcycle_copy", C.c_int32), ("local_build", C.c_int32)]


FIELD_FN = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                       C.c_void_p)

_lib = None


def load():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2009_13840_amd.build`")
    # torch first: the library then binds to the HIP runtime torch already loaded
    # (both carry the soname libamdhip64.so.7), so one runtime serves the process.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int, C.POINTER(C.c_double)
    sig = {
        "hho_last_error": ([], C.c_char_p),
        "hho_options_default": ([C.POINTER(Options)], None),
        "hho_mesh_create": ([C.POINTER(MeshDesc), C.POINTER(P)], I32),
        "hho_mesh_destroy": ([P], None),
        "hho_problem_create": ([P, I32, I32, I32, C.POINTER(C.c_int), C.POINTER(Options), C.POINTER(P)], I32),
        "hho_problem_destroy": ([P], None),
        "hho_problem_set_data": ([P, FIELD_FN, FIELD_FN, FIELD_FN, P], I32),
        "hho_workspace_size": ([P, C.POINTER(C.c_size_t)], I32),
        "hho_bind_workspace": ([P, P, C.c_size_t], I32),
        "hho_set_stream": ([P, P], I32),
        "hho_set_graph": ([P, I32], I32),
        "hho_setup": ([P], I32),
        "hho_level_size": ([P, I32, C.POINTER(I64)], I32),
        "hho_solve": ([P, D, I64, D, I64, C.POINTER(C.c_int), D, I32, D], I32),
        "hho_solve_device": ([P, P, C.POINTER(C.c_int), D, I32, D], I32),
        "hho_solution_sizes": ([P, C.POINTER(I64), C.POINTER(I64)], I32),
        "hho_moments_size": ([P, C.POINTER(I64), C.POINTER(I64)], I32),
        "hho_set_moments": ([P, D, D], I32),
        "hho_batch_create": ([C.POINTER(P), I32, C.POINTER(P)], I32),
        "hho_batch_destroy": ([P], None),
        "hho_batch_problem": ([P, C.POINTER(P)], I32),
        "hho_batch_sizes": ([P, C.POINTER(I64), C.POINTER(I64)], I32),
        "hho_batch_solve": ([P, D, C.POINTER(I64), D, C.POINTER(I64), C.POINTER(C.c_int), D, C.POINTER(I64), D,
                             C.POINTER(C.c_int)], I32),
        "hho_learned_save": ([P, P, C.c_size_t, C.POINTER(C.c_size_t)], I32),
        "hho_learned_load": ([P, P, C.c_size_t], I32),
        "hho_get_rhs": ([P, P], I32),
        "hho_recover_cells": ([P, P, P, P], I32),
        "hho_get_condensed_cell": ([P, I64, D, D, I64, C.POINTER(I64)], I32),
        "hho_get_local_cell": ([P, I64, D, D, D, D, I64, C.POINTER(I64)], I32),
        "hho_local_hp_cell": ([P, C.c_int, C.c_double, C.c_int, I64, FIELD_FN, FIELD_FN, FIELD_FN, P, D, D, D, D,
                               I64, C.POINTER(I64), C.POINTER(I64)], I32),
        "hho_hp_skeleton": ([P, C.c_int, C.c_double, C.c_int, FIELD_FN, FIELD_FN, FIELD_FN, P, P, P, D, D, I64,
                             C.POINTER(I64), C.POINTER(I64)], I32),
        "hho_level_apply": ([P, I32, P, P], I32),
        "hho_precond_apply": ([P, I32, P, P], I32),
        "hho_vcycle_level_apply": ([P, I32, I32, P, P], I32),
        "hho_vcycle_apply": ([P, P, P], I32),
        "hho_get_timings": ([P, D, I32], I32),
        "hho_upload": ([P], I32),
        "hho_time_kernel": ([P, I32, I32, I32, D], I32),
        "hho_coarse_prec_apply": ([P, P, P], I32),
        "hho_coarse_solve_apply": ([P, P, P], I32),
        "hho_direct_info": ([P, C.c_char_p, P, C.c_int64, P], I32),
        "hho_debug_copy": ([P, C.c_char_p, I32, D, I64, C.POINTER(I64)], I32),
        "hho_mesh_create_union": ([C.POINTER(MeshDesc), I32, C.POINTER(P), C.POINTER(I64), C.POINTER(I64)], I32),
        "hho_problem_set_segments": ([P, I32, C.POINTER(I64), C.POINTER(I64)], I32),
        "hho_batch_results": ([P, C.POINTER(C.c_int), D, I32], I32),
        "hho_autotune": ([P, I32, C.POINTER(C.c_int)], I32),
        "hho_learned_dims": ([P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(I64)], I32),
        "hho_learned_set_params": ([P, C.POINTER(C.c_float), I64], I32),
        "hho_learned_get_params": ([P, C.POINTER(C.c_float), I64], I32),
        "hho_learned_enable": ([P, I32], I32),
        "hho_learned_apply": ([P, P, P], I32),
        "hho_learned_collect": ([P, P, I32, P, P, I64, C.POINTER(I64)], I32),
        "hho_learned_grad": ([P, P, P, I64, C.POINTER(C.c_float), D], I32),
        "hho_learned_grad_noalloc": ([P, P, P, I64, C.POINTER(C.c_float), D], I32),
        "hho_set_tolerances": ([P, C.c_double, I32, C.c_double, I32], I32),
        "hho_probe_arm": ([P, C.c_uint, I32], I32),
        "hho_probe_read": ([P, I32, I32, C.POINTER(I64), D, C.POINTER(I64)], I32),
        "hho_probe_clear": ([P], I32),
        "hho_amg_level_info": ([P, I32, C.POINTER(I64)], I32),
        "hho_learned_train": ([P, P, P, I64, I32, I32, C.c_float, C.c_uint64, C.POINTER(C.c_float)], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(code):
    if code != HHO_OK:
        raise HHOError(code, load().hho_last_error().decode())
    return code


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _desc(m):
    keep = [np.ascontiguousarray(m.verts, dtype=np.float64),
            np.ascontiguousarray(m.face_ptr, dtype=np.int64),
            np.ascontiguousarray(m.face_vtx, dtype=np.int64),
            np.ascontiguousarray(m.cell_ptr, dtype=np.int64),
            np.ascontiguousarray(m.cell_face, dtype=np.int64),
            np.ascontiguousarray(m.face_bc, dtype=np.int8)]
    v, fp, fv, cp, cf, bc = keep
    desc = MeshDesc(int(m.dim), len(v), _dptr(v), len(fp) - 1, fp.ctypes.data_as(C.POINTER(C.c_int64)),
                    fv.ctypes.data_as(C.POINTER(C.c_int64)), len(cp) - 1,
                    cp.ctypes.data_as(C.POINTER(C.c_int64)), cf.ctypes.data_as(C.POINTER(C.c_int64)),
                    bc.ctypes.data_as(C.POINTER(C.c_int8)))
    return desc, keep


class Mesh:
    """Library copy of a ``synth.Mesh``-like object (dim, verts, face_ptr, face_vtx,
    cell_ptr, cell_face, face_bc)."""

    def __init__(self, m):
        lib = load()
        desc, keep = _desc(m)
        self._keep = keep
        h = C.c_void_p()
        _check(lib.hho_mesh_create(C.byref(desc), C.byref(h)))
        self.h = h
        self.dim = int(m.dim)
        self.n_faces = len(keep[1]) - 1
        self.n_cells = len(keep[3]) - 1

    def local_hp_cell(self, k: int, cell: int, f=None, gD=None, gN=None, eta: float = 1.0, qdeg=None):
        """The HHO-hp scheme's local operators of one cell (hho_local_hp_cell)."""
        lib = load()
        d = self.dim
        cbs = (_wrap_field(f, d, False), _wrap_field(gD, d, False), _wrap_field(gN, d, True))
        qdeg = 2 * k + 8 if qdeg is None else qdeg
        nloc, npl = C.c_int64(), C.c_int64()
        st = lib.hho_local_hp_cell(self.h, k, eta, qdeg, cell, *cbs, None, None, None, None, None, 0,
                                   C.byref(nloc), C.byref(npl))
        if st not in (0, -7):
            _check(st)
        n, m = nloc.value, npl.value
        cap = max(n * n, d * m * n)
        a, B, ru, rp = np.zeros(cap), np.zeros(cap), np.zeros(d * n), np.zeros(m)
        _check(lib.hho_local_hp_cell(self.h, k, eta, qdeg, cell, *cbs, None, _dptr(a), _dptr(B), _dptr(ru),
                                     _dptr(rp), cap, C.byref(nloc), C.byref(npl)))
        return {"a": a[:n * n].reshape(n, n).copy(), "B": B[:d * m * n].reshape(d, m, n).copy(),
                "rhs_u": ru.reshape(d, n).copy(), "rhs_p": rp.copy()}

    def hp_skeleton(self, k: int, f=None, gD=None, gN=None, eta: float = 1.0, qdeg=None):
        """The HHO-hp scheme's v&p-cond skeleton (hho_hp_skeleton): a scipy CSR
        matrix and its right-hand side."""
        import scipy.sparse as sp
        lib = load()
        d = self.dim
        cbs = (_wrap_field(f, d, False), _wrap_field(gD, d, False), _wrap_field(gN, d, True))
        qdeg = 2 * k + 8 if qdeg is None else qdeg
        n, nnz = C.c_int64(), C.c_int64()
        st = lib.hho_hp_skeleton(self.h, k, eta, qdeg, *cbs, None, None, None, None, None, 0, C.byref(n), C.byref(nnz))
        if st not in (0, -7):
            _check(st)
        rp = np.zeros(n.value + 1, dtype=np.int64)
        ci = np.zeros(nnz.value, dtype=np.int64)
        v, b = np.zeros(nnz.value), np.zeros(n.value)
        _check(lib.hho_hp_skeleton(self.h, k, eta, qdeg, *cbs, None, rp.ctypes.data_as(C.c_void_p),
                                   ci.ctypes.data_as(C.c_void_p), _dptr(v), _dptr(b), nnz.value,
                                   C.byref(n), C.byref(nnz)))
        return sp.csr_matrix((v, ci, rp), shape=(n.value, n.value)), b

    @classmethod
    def union(cls, meshes):
        """Disjoint union of several meshes; returns (mesh, face_offsets, cell_offsets)."""
        lib = load()
        pairs = [_desc(m) for m in meshes]
        arr = (MeshDesc * len(pairs))(*[d for d, _ in pairs])
        fo = np.zeros(len(pairs) + 1, dtype=np.int64)
        co = np.zeros(len(pairs) + 1, dtype=np.int64)
        h = C.c_void_p()
        _check(lib.hho_mesh_create_union(arr, len(pairs), C.byref(h), fo.ctypes.data_as(C.POINTER(C.c_int64)),
                                         co.ctypes.data_as(C.POINTER(C.c_int64))))
        self = cls.__new__(cls)
        self._keep = []
        self.h = h
        self.dim = int(meshes[0].dim)
        self.n_faces = int(fo[-1])
        self.n_cells = int(co[-1])
        return self, fo, co

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hho_mesh_destroy(self.h)
            self.h = None


def options(**kw) -> Options:
    o = Options()
    load().hho_options_default(C.byref(o))
    names = {f[0] for f in Options._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown option {k!r}; known: {sorted(names)}")
        if k == "precision":
            v = PREC[v] if isinstance(v, str) else v
        if k == "coarse_mode":
            v = COARSE[v] if isinstance(v, str) else v
        if k == "vcycle_copy":
            v = COPY[v] if isinstance(v, str) else v
        if k == "local_build":
            v = LOCAL[v] if isinstance(v, str) else v
        if k == "smoother":
            v = SMOOTHER[v] if isinstance(v, str) else v
        setattr(o, k, v)
    return o


def _wrap_field(fn, dim, with_normal):
    if fn is None:
        return FIELD_FN()

    def cb(x, n, nrm, out, ctx):
        try:
            X = np.ctypeslib.as_array(x, shape=(n * dim,)).reshape(n, dim)
            O = np.ctypeslib.as_array(out, shape=(n * dim,)).reshape(n, dim)
            if with_normal:
                N = np.ctypeslib.as_array(nrm, shape=(n * dim,)).reshape(n, dim)
                O[:] = fn(X, N)
            else:
                O[:] = fn(X)
        except Exception as e:  # pragma: no cover - surfaces in the caller
            print("hho field callback failed:", repr(e))
            O[:] = np.nan
    return FIELD_FN(cb)


class Problem:
    def __init__(self, mesh: Mesh, k: int, cond: str = "v", degrees=None, **opts):
        lib = load()
        self.mesh = mesh
        self.k, self.cond = k, cond
        self.opts = options(**opts)
        h = C.c_void_p()
        if degrees is None:
            degp, nlev = None, 0
        else:
            arr = (C.c_int * len(degrees))(*degrees)
            degp, nlev = arr, len(degrees)
        _check(lib.hho_problem_create(mesh.h, k, COND[cond], nlev, degp, C.byref(self.opts), C.byref(h)))
        self.h = h
        self.ws = None
        self.nlev = len(degrees) if degrees is not None else k + 1
        self.nfaces = mesh.n_faces

    def __del__(self):
        # a batch's combined problem belongs to the batch (hho_batch_destroy frees it)
        if getattr(self, "h", None) and _lib is not None and not getattr(self, "_borrowed", False):
            _lib.hho_problem_destroy(self.h)
            self.h = None

    # ---- host phase
    def set_data(self, f=None, gD=None, gN=None):
        d = self.mesh.dim
        self._cbs = (_wrap_field(f, d, False), _wrap_field(gD, d, False), _wrap_field(gN, d, True))
        _check(load().hho_problem_set_data(self.h, *self._cbs, None))

    def local_cell(self, c: int):
        lib = load()
        nloc = C.c_int64()
        cap = 1 << 16
        d = self.mesh.dim
        a = np.zeros(cap)
        B = np.zeros(cap)
        ru = np.zeros(cap)
        rp = np.zeros(cap)
        _check(lib.hho_get_local_cell(self.h, c, _dptr(a), _dptr(B), _dptr(ru), _dptr(rp), cap, C.byref(nloc)))
        n = nloc.value
        from math import comb
        nT = comb(self.k + d, d)
        return {"a": a[:n * n].reshape(n, n).copy(), "B": B[:d * nT * n].reshape(d, nT, n).copy(),
                "rhs_u": ru[:d * n].reshape(d, n).copy(), "rhs_p": rp[:nT].copy()}

    def set_graph(self, on: bool = True):
        """Replay every V-cycle from a captured HIP graph (hho_set_graph)."""
        _check(load().hho_set_graph(self.h, 1 if on else 0))

    def workspace_size(self) -> int:
        s = C.c_size_t()
        _check(load().hho_workspace_size(self.h, C.byref(s)))
        return s.value

    # ---- device phase
    def bind(self, device="cuda:0", fill=None):
        """Allocate the workspace (optionally every byte set to `fill`) and bind it."""
        import torch
        n = self.workspace_size()
        if fill is None:
            self.ws = torch.empty(n, dtype=torch.uint8, device=device)
        else:
            self.ws = torch.full((n,), fill, dtype=torch.uint8, device=device)
        _check(load().hho_bind_workspace(self.h, C.c_void_p(self.ws.data_ptr()), n))
        stream = torch.cuda.current_stream(self.ws.device).cuda_stream
        _check(load().hho_set_stream(self.h, C.c_void_p(stream)))
        self.device = self.ws.device

    def upload(self):
        _check(load().hho_upload(self.h))

    def setup(self):
        _check(load().hho_setup(self.h))

    def time_kernel(self, kind: int, level: int = 0, reps: int = 20) -> float:
        ms = C.c_double()
        _check(load().hho_time_kernel(self.h, kind, level, reps, C.byref(ms)))
        return ms.value

    def set_tolerances(self, rtol, max_it=1000, coarse_rtol=1e-3, coarse_max_it=300):
        _check(load().hho_set_tolerances(self.h, rtol, max_it, coarse_rtol, coarse_max_it))

    # ---- live kernel timing
    def probe_arm(self, mask: int, stride: int = 1):
        _check(load().hho_probe_arm(self.h, mask, stride))

    def probe_clear(self):
        _check(load().hho_probe_clear(self.h))

    def probe_read(self, kind: int, level: int = -1):
        """(timed launches, their total ms, all launches) of the armed class
        `kind` on `level` (-1: all levels)."""
        n, ms, alln = C.c_int64(), C.c_double(), C.c_int64()
        _check(load().hho_probe_read(self.h, kind, level, C.byref(n), C.byref(ms), C.byref(alln)))
        return n.value, ms.value, alln.value

    def amg_level_info(self, level: int):
        info = (C.c_int64 * 7)()
        _check(load().hho_amg_level_info(self.h, level, info))
        keys = ("n", "nc", "nnz_a", "nnz_p", "nnz_b", "explicit_from", "levels")
        return dict(zip(keys, list(info)))

    def level_size(self, l: int) -> int:
        n = C.c_int64()
        _check(load().hho_level_size(self.h, l, C.byref(n)))
        return n.value

    def _vec(self, n):
        import torch
        return torch.zeros(n, dtype=torch.float64, device=self.device)

    def solve(self, hist_cap: int = 1001):
        x = self._vec(self.level_size(0))
        it = C.c_int()
        hist = np.zeros(hist_cap)
        rel = C.c_double()
        code = load().hho_solve_device(self.h, C.c_void_p(x.data_ptr()), C.byref(it), _dptr(hist), hist_cap,
                                C.byref(rel))
        if code not in (HHO_OK, -4):
            _check(code)
        n = min(it.value + 1, hist_cap)
        return x, it.value, hist[:n].copy(), rel.value, code == HHO_OK

    def solution_sizes(self):
        fn, pn = C.c_int64(), C.c_int64()
        _check(load().hho_solution_sizes(self.h, C.byref(fn), C.byref(pn)))
        return fn.value, pn.value

    def solve_host(self, face_cap=None, p_cap=None, hist_cap: int = 1001):
        """hho_solve into host arrays: (face modes, cell pressure modes, iterations,
        residual history, final relative residual, converged)."""
        fn, pn = self.solution_sizes()
        face = np.zeros(fn if face_cap is None else face_cap)
        pres = np.zeros(pn if p_cap is None else p_cap)
        it = C.c_int()
        hist = np.zeros(hist_cap)
        rel = C.c_double()
        code = load().hho_solve(self.h, _dptr(face), face.size, _dptr(pres), pres.size, C.byref(it), _dptr(hist),
                                hist_cap, C.byref(rel))
        if code not in (HHO_OK, -4):
            _check(code)
        n = min(it.value + 1, hist_cap)
        return face[:fn], pres[:pn], it.value, hist[:n].copy(), rel.value, code == HHO_OK

    def moments_size(self):
        nu, npp = C.c_int64(), C.c_int64()
        _check(load().hho_moments_size(self.h, C.byref(nu), C.byref(npp)))
        return nu.value, npp.value

    def set_moments(self, rhs_u, rhs_p):
        nu, npp = self.moments_size()
        ru = np.ascontiguousarray(rhs_u, dtype=np.float64)
        rp = np.ascontiguousarray(rhs_p, dtype=np.float64)
        if ru.size != nu or rp.size != npp:
            raise ValueError(f"set_moments: need {nu} and {npp} values, got {ru.size} and {rp.size}")
        _check(load().hho_set_moments(self.h, _dptr(ru), _dptr(rp)))

    def learned_save(self) -> bytes:
        need = C.c_size_t()
        code = load().hho_learned_save(self.h, None, 0, C.byref(need))
        if code != -7:
            _check(code)
        buf = C.create_string_buffer(need.value)
        _check(load().hho_learned_save(self.h, C.cast(buf, C.c_void_p), need.value, C.byref(need)))
        return buf.raw

    def learned_load(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        _check(load().hho_learned_load(self.h, C.cast(buf, C.c_void_p), len(data)))

    def rhs(self):
        b = self._vec(self.level_size(0))
        _check(load().hho_get_rhs(self.h, C.c_void_p(b.data_ptr())))
        return b

    def recover_cells(self, x):
        """Cell velocities [n_cells, d*n_T] and full cell pressures [n_cells, n_T]
        (device tensors) from the level-0 solution x."""
        import torch
        from math import comb
        d = self.mesh.dim
        nT = comb(self.k + d, d)
        nc = self.mesh.n_cells
        assert x.dtype == torch.float64 and x.is_contiguous() and x.numel() == self.level_size(0)
        u = torch.empty((nc, d * nT), dtype=torch.float64, device=x.device)
        p = torch.empty((nc, nT), dtype=torch.float64, device=x.device)
        _check(load().hho_recover_cells(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(u.data_ptr()),
                                        C.c_void_p(p.data_ptr())))
        return u, p

    def condensed_cell(self, c: int):
        n = C.c_int64()
        cap = 1 << 18
        S = np.zeros(cap)
        r = np.zeros(4096)
        _check(load().hho_get_condensed_cell(self.h, c, _dptr(S), _dptr(r), cap, C.byref(n)))
        m = n.value
        return S[:m * m].reshape(m, m).copy(), r[:m].copy()

    def level_apply(self, l, x):
        y = self._vec(self.level_size(l))
        _check(load().hho_level_apply(self.h, l, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())))
        return y

    def vcycle_level_apply(self, l, x, which: int = 0):
        """y = S_l x (which 0) or M_l x (which 1) in the V-cycle's precision."""
        y = self._vec(self.level_size(l))
        _check(load().hho_vcycle_level_apply(self.h, l, which, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())))
        return y

    def precond_apply(self, l, r):
        z = self._vec(self.level_size(l))
        _check(load().hho_precond_apply(self.h, l, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr())))
        return z

    def debug_copy(self, name: str, level: int = 0):
        n = C.c_int64()
        out = np.zeros(1 << 22)
        _check(load().hho_debug_copy(self.h, name.encode(), level, _dptr(out), out.size, C.byref(n)))
        return out[:n.value].copy()

    def coarse_prec_apply(self, v):
        z = self._vec(self.level_size(self.nlev - 1))
        _check(load().hho_coarse_prec_apply(self.h, C.c_void_p(v.data_ptr()), C.c_void_p(z.data_ptr())))
        return z

    def direct_info(self, name: str):
        """The sparse direct coarse solver's symbolic arrays (hho_direct_info)."""
        n = C.c_int64()
        st = load().hho_direct_info(self.h, name.encode(), None, 0, C.byref(n))
        if st != -7:
            _check(st)
        out = np.zeros(max(n.value, 1), dtype=np.int64)
        _check(load().hho_direct_info(self.h, name.encode(), out.ctypes.data_as(C.c_void_p), out.size, C.byref(n)))
        return out[:n.value].copy()

    def coarse_solve_apply(self, b):
        x = self._vec(self.level_size(self.nlev - 1))
        _check(load().hho_coarse_solve_apply(self.h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr())))
        return x

    def vcycle_apply(self, b):
        x = self._vec(self.level_size(0))
        _check(load().hho_vcycle_apply(self.h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr())))
        return x

    def autotune(self, reps=10):
        """Fastest launch shapes per level (operator block, patch threads); re-runs setup."""
        ch = np.zeros(2 * self.nlev, dtype=np.int32)
        _check(load().hho_autotune(self.h, reps, ch.ctypes.data_as(C.POINTER(C.c_int))))
        self.setup()
        return ch.reshape(-1, 2)

    # ---- batches (problem on a union mesh)
    def set_segments(self, face_ptr, cell_ptr):
        fp = np.ascontiguousarray(face_ptr, dtype=np.int64)
        cp = np.ascontiguousarray(cell_ptr, dtype=np.int64)
        self.nseg = len(fp) - 1
        _check(load().hho_problem_set_segments(self.h, self.nseg, fp.ctypes.data_as(C.POINTER(C.c_int64)),
                                               cp.ctypes.data_as(C.POINTER(C.c_int64))))

    def batch_results(self):
        its = np.zeros(self.nseg, dtype=np.int32)
        rel = np.zeros(self.nseg)
        _check(load().hho_batch_results(self.h, its.ctypes.data_as(C.POINTER(C.c_int)), _dptr(rel), self.nseg))
        return its, rel

    # ---- learned fine-level smoother (problem created with learned=1)
    def learned_dims(self):
        a, b, c, n = C.c_int(), C.c_int(), C.c_int(), C.c_int64()
        _check(load().hho_learned_dims(self.h, C.byref(a), C.byref(b), C.byref(c), C.byref(n)))
        return dict(n_in=a.value, n_out=b.value, hidden=c.value, n_params=n.value)

    def learned_set_params(self, prm):
        prm = np.ascontiguousarray(prm, dtype=np.float32)
        _check(load().hho_learned_set_params(self.h, prm.ctypes.data_as(C.POINTER(C.c_float)), prm.size))

    def learned_get_params(self):
        out = np.zeros(self.learned_dims()["n_params"], dtype=np.float32)
        _check(load().hho_learned_get_params(self.h, out.ctypes.data_as(C.POINTER(C.c_float)), out.size))
        return out

    def learned_enable(self, on=True):
        _check(load().hho_learned_enable(self.h, 1 if on else 0))

    def learned_apply(self, r):
        z = self._vec(self.level_size(0))
        _check(load().hho_learned_apply(self.h, C.c_void_p(r.data_ptr()), C.c_void_p(z.data_ptr())))
        return z

    def learned_collect(self, x_true, cycles):
        import torch
        dm = self.learned_dims()
        cap = cycles * self.nfaces
        X = torch.zeros((cap, dm["n_in"]), dtype=torch.float32, device=self.device)
        T = torch.zeros((cap, dm["n_out"]), dtype=torch.float32, device=self.device)
        n = C.c_int64()
        _check(load().hho_learned_collect(self.h, C.c_void_p(x_true.data_ptr()), cycles, C.c_void_p(X.data_ptr()),
                                          C.c_void_p(T.data_ptr()), cap, C.byref(n)))
        return X[:n.value], T[:n.value]

    def learned_grad(self, X, T, noalloc=False):
        """Loss and parameter gradient over the rows of X, T (device FP32);
        noalloc=True calls the variant whose work arrays live in the library's
        fixed device array instead of the workspace."""
        g = np.zeros(self.learned_dims()["n_params"], dtype=np.float32)
        loss = C.c_double()
        fn = load().hho_learned_grad_noalloc if noalloc else load().hho_learned_grad
        _check(fn(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()), X.shape[0],
                  g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss)))
        return loss.value, g

    def learned_train(self, X, T, steps, batch=1024, lr=1e-3, seed=0):
        hist = np.zeros(steps, dtype=np.float32)
        _check(load().hho_learned_train(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()), X.shape[0],
                                        steps, batch, lr, seed, hist.ctypes.data_as(C.POINTER(C.c_float))))
        return hist

    def timings(self):
        t = np.zeros(16)
        _check(load().hho_get_timings(self.h, _dptr(t), 16))
        keys = ["condense_ms", "assemble_ms", "levels_ms", "smoother_setup_ms", "coarse_setup_ms", "solve_ms",
                "vcycle_ms", "vcycles", "coarse_its", "local_ms"]
        return dict(zip(keys, t[:len(keys)]))


class Batch:
    """hho_batch_create over separately created problems (each after set_data);
    ``problem`` is the combined problem to bind, set up and time."""

    def __init__(self, problems):
        lib = load()
        arr = (C.c_void_p * len(problems))(*[q.h for q in problems])
        h = C.c_void_p()
        _check(lib.hho_batch_create(arr, len(problems), C.byref(h)))
        self.h = h
        self.n = len(problems)
        ph = C.c_void_p()
        _check(lib.hho_batch_problem(self.h, C.byref(ph)))
        P = Problem.__new__(Problem)
        P.h, P.mesh, P.k, P.cond, P.ws = ph, problems[0].mesh, problems[0].k, problems[0].cond, None
        P.nlev, P.opts, P._owner = problems[0].nlev, problems[0].opts, self
        P._borrowed = True
        P.nfaces = None
        self.problem = P

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hho_batch_destroy(self.h)
            self.h = None

    def sizes(self):
        fn = np.zeros(self.n, dtype=np.int64)
        pn = np.zeros(self.n, dtype=np.int64)
        _check(load().hho_batch_sizes(self.h, fn.ctypes.data_as(C.POINTER(C.c_int64)),
                                      pn.ctypes.data_as(C.POINTER(C.c_int64))))
        return fn, pn

    def solve(self, hist_cap: int = 200):
        """Per member: (face modes, cell pressure modes, iterations, history,
        final relative residual, status)."""
        fn, pn = self.sizes()
        foff = np.concatenate([[0], np.cumsum(fn)]).astype(np.int64)
        poff = np.concatenate([[0], np.cumsum(pn)]).astype(np.int64)
        hoff = (np.arange(self.n + 1) * hist_cap).astype(np.int64)
        face = np.zeros(int(foff[-1]))
        pres = np.zeros(int(poff[-1]))
        its = np.zeros(self.n, dtype=np.int32)
        hist = np.full(int(hoff[-1]), np.nan)
        rel = np.zeros(self.n)
        st = np.zeros(self.n, dtype=np.int32)
        i64 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))  # noqa: E731
        i32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))  # noqa: E731
        code = load().hho_batch_solve(self.h, _dptr(face), i64(foff), _dptr(pres), i64(poff), i32(its), _dptr(hist),
                                      i64(hoff), _dptr(rel), i32(st))
        if code not in (HHO_OK, -4):
            _check(code)
        out = []
        for i in range(self.n):
            h = hist[hoff[i]:hoff[i + 1]]
            out.append((face[foff[i]:foff[i + 1]], pres[poff[i]:poff[i + 1]], int(its[i]),
                        h[~np.isnan(h)], float(rel[i]), int(st[i])))
        return out

