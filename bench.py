"""Benchmark: one step = the whole hot path on one synthetic problem --
static condensation of every cell, assembly of the face-block operator,
inheritance of the coarse levels k-1..0, smoother-patch and coarse-solver
setup, and the FGMRES + p-multilevel V-cycle solve to a 1e-8 relative residual.
Inputs (mesh topology and local HHO operators) are resident in device memory
before the timed region starts.

Default workload: 2D Lloyd-relaxed Voronoi mesh of the unit square with 16384
cells, HHO degree k = 3 (face block 2(k+1) = 8), v-cond, V-cycle 3->2->1->0,
seeded trig-series body force, homogeneous Dirichlet boundary, FP64.

Prints one JSON line (see the metric/roofline/cpu_baseline fields).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8 residual & V-cycle GDOF/s: mixed/learned vs plain FP64, 1 GPU"
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
PROBE_STRIDE = 11  # prime: the samples cycle through every position of the solver's periodic launch pattern


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("k_spmv.hip", "k_solve.hip", "k_amg.hip", "device.h", "dev_common.h"):
        with open(os.path.join(ROOT, "paper_2009_13840_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by the plain-copy factor), or
    None when no summary exists or the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get(workload, {}).get(kernel)
    if not ent or ent.get("source_digest") != kernel_source_digest():
        return None
    return ent["bytes_per_launch"]


WORKLOADS = {
    "voronoi16384_k3_v": dict(mesh="voronoi", n=16384, seed=2, k=3, cond="v"),
    "voronoi16384_k3_vp": dict(mesh="voronoi", n=16384, seed=2, k=3, cond="vp"),
    "quad8_k1_v": dict(mesh="quad", n=8, seed=1, k=1, cond="v"),
    # unit cube, uniform hexahedra, homogeneous Dirichlet, trig-series force
    "hex32_k2_vp": dict(mesh="hex", n=32, seed=3, k=2, cond="vp"),
    "hex32_k3_vp": dict(mesh="hex", n=32, seed=3, k=3, cond="vp"),
    "hex24_k3_v": dict(mesh="hex", n=24, seed=1000, k=3, cond="v"),
}


def make_mesh(spec):
    from synth import voronoi_lloyd, cartesian_quads, cartesian_hexes
    if spec["mesh"] == "voronoi":
        return voronoi_lloyd(spec["n"], spec["seed"])
    if spec["mesh"] == "quad":
        return cartesian_quads(spec["n"])
    return cartesian_hexes(spec["n"])


def make_data(spec, dim):
    from synth import trig_series, stokes_sincos_2d
    from synth.fields import problem_data
    if spec["mesh"] == "quad":
        return problem_data(stokes_sincos_2d(), None, dim)
    return problem_data(None, trig_series(dim, spec["seed"]), dim)


def spmv_bytes(mesh, k, cond, level_k, dtype_bytes=8, value_bytes=None):
    """Algorithmic bytes of one application of the level operator: every stored
    value once (value_bytes each, default the vectors' dtype_bytes), the int32
    block structure, x read once and y written once."""
    from math import comb
    d = mesh.dim
    p = comb(level_k + d - 1, d - 1)
    t = comb(level_k + d, d) if cond == "v" else 1
    bs = p if cond == "v" else d * p
    cptr = np.asarray(mesh.cell_ptr)
    nfc = np.diff(cptr)
    fc = mesh.face_cells()
    # face stencil rows: faces of the cells sharing each face
    nnzb = 0
    for f in range(mesh.n_faces):
        cells = fc[f][fc[f] >= 0]
        nnzb += int(sum(nfc[c] for c in cells) - (len(cells) - 1))
    ncf = int(cptr[-1])
    vals = nnzb * bs * bs + ncf * d * p * (t if cond == "v" else 1) + (mesh.n_cells * t * t if cond == "v" else 0)
    N = mesh.n_faces * d * p + mesh.n_cells * t
    idx = 4 * (nnzb + mesh.n_faces + 1 + ncf + mesh.n_cells + 1 + 4 * mesh.n_faces)
    vb = dtype_bytes if value_bytes is None else value_bytes
    return vals * vb + idx + 2 * N * dtype_bytes, dict(nnzb=nnzb, N=N, values=vals)


def precond_bytes(mesh, k, cond, dtype_bytes=8):
    """Algorithmic bytes of one cell-patch Schwarz application on the level of
    degree k: per cell the packed patch inverse (n (n + 1) / 2 values, n = the
    patch's face rows of one component block), the pressure coupling and its
    Schur data, the residual of the patch read and the corrections written once."""
    from math import comb
    d = mesh.dim
    p = comb(k + d - 1, d - 1)
    t = comb(k + d, d)
    nfc = np.diff(np.asarray(mesh.cell_ptr)).astype(np.int64)
    if cond == "v":
        m = nfc * p
        vals = m * (m + 1) // 2 + nfc * d * p * t + t * t
        io = 2 * (nfc * d * p + t)
    else:
        n = nfc * d * p
        vals = n * (n + 1) // 2 + n + nfc * d * p + 1
        io = 2 * (n + 1)
    idx = 4 * (int(nfc.sum()) * 3 + 2 * mesh.n_cells)
    return int((vals + io).sum()) * dtype_bytes + idx


def precond_kernel_name(mesh, k, cond):
    from math import comb
    d = mesh.dim
    p = comb(k + d - 1, d - 1)
    rows = int(np.diff(np.asarray(mesh.cell_ptr)).max()) * (p if cond == "v" else d * p)
    return f"k_precond<double, {(rows + 63) // 64}, {d if cond == 'v' else 1}>"


STORAGE_TYPES = {"fp64": "double, double, double", "fp32": "float, float, float", "bf16": "float, hho::bf16, float"}


def fine_kernel_name(d, k, cond, precision):
    """Name of a level's operator kernel in its V-cycle (two-slot input) form, as
    rocprofv3 lists it (arithmetic type, operator storage, smoother storage)."""
    from math import comb
    T = STORAGE_TYPES[precision]
    p = comb(k + d - 1, d - 1)
    if cond == "v":
        return f"k_spmv_v<{T}, {d}, {p}, {comb(k + d, d)}, true, 0>"
    return f"k_spmv_vp<{T}, {d * p}, true, 0>"


def train_learned(P, n0, forcings=200, cycles=3, steps=1500, batch=2048, lr=1e-3):
    """Untimed: V-cycle training pairs from 200 seeded discrete forcings
    b = S x_true (x_true ~ N(0, 1) per unknown from seeds 0..199; the solve that
    is timed afterwards uses the workload's body force, which the network never
    saw), He-uniform first layer and zero output layer, Adam training on the GPU
    by the library's kernels."""
    import torch
    dm = P.learned_dims()
    rng = np.random.default_rng(0)
    h, n_in, n_out = dm["hidden"], dm["n_in"], dm["n_out"]
    W1 = (2 * rng.random(h * n_in) - 1) * np.sqrt(6.0 / n_in)
    W2 = np.zeros(n_out * h)  # the untrained network is the zero predictor
    P.learned_set_params(np.concatenate([W1, np.zeros(h), W2, np.zeros(n_out)]).astype(np.float32))
    P.setup()
    t0 = time.perf_counter()
    Xs, Ts = [], []
    for i in range(forcings):
        xt = torch.from_numpy(np.random.default_rng(i).standard_normal(n0)).cuda()
        X, T = P.learned_collect(xt, cycles)
        Xs.append(X)
        Ts.append(T)
    X, T = torch.cat(Xs), torch.cat(Ts)
    del Xs, Ts
    base = float(0.5 * (T.double() ** 2).sum(dim=1).mean())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = P.learned_train(X, T, steps=steps, batch=batch, lr=lr, seed=7)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    npairs = int(X.shape[0])
    del X, T
    torch.cuda.empty_cache()
    P.setup()
    _, its_plain, _, _, _ = P.solve()
    P.learned_enable(True)
    print(f"[bench] learned smoother: {npairs} pairs from {forcings} forcings ({t1 - t0:.1f}s), {steps} Adam steps "
          f"({t2 - t1:.1f}s), loss {hist[:10].mean():.3e} -> {hist[-50:].mean():.3e} (zero predictor {base:.3e})",
          file=sys.stderr, flush=True)
    return {"pairs": npairs, "forcings": forcings, "forcing_seeds": f"0..{forcings - 1}", "collect_s": round(t1 - t0, 2),
            "train_steps": steps, "batch": batch, "train_s": round(t2 - t1, 2),
            "loss_first": float(hist[:10].mean()), "loss_last": float(hist[-50:].mean()),
            "loss_zero_predictor": base, "fgmres_its_plain": its_plain,
            "network": "bfloat16 weights and activations, FP32 sums on the matrix cores; "
                       f"{n_in} inputs, {h} hidden, {n_out} outputs (face velocity and both cells' pressures)"}


_POOL_INPUT = None  # (mesh, geo, eta, data) of the CPU baseline, inherited by forked workers


def _oracle_local(cells):
    """Worker of the untimed host phase of the CPU baseline: the oracle's local
    operators of some cells (the same call its build step makes)."""
    from oracle.hho import local_hho
    mesh, geo, eta, data = _POOL_INPUT
    return [local_hho(mesh, geo, c, eta, *data) for c in cells]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec, sample_cells=4096, coarse="amg"):
    """The oracle as it stands, on a bounded sample of the workload's family (the
    same mesh generator and seed, fewer cells; same degree, variant and solver
    settings: cell-patch Schwarz GMRES(2) smoothing, coarsest level by GMRES to
    1e-2 (2D) or 1e-3 (3D) with the block-triangular AMG preconditioner, FGMRES
    to 1e-8).  Timed:
    the phases of the GPU step -- condensation, assembly, coarse operators,
    smoother and coarse-solver setup, FGMRES.  Untimed: the mesh and the local
    HHO operators (the GPU step takes them as input too), the latter spread over
    a process pool.  Reported in the metric's unit, fine DOFs solved per second."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    from threadpoolctl import threadpool_info
    import oracle.solve as OS
    from oracle.hho import mesh_geometry
    from oracle.condense import condense_v, condense_vp
    from oracle.system import assemble_condensed, coarse_indices, layout, nullspace
    from synth import voronoi_lloyd, cartesian_hexes
    if spec["mesh"] == "voronoi":
        mesh = voronoi_lloyd(sample_cells, spec["seed"])
        name = f"voronoi{sample_cells}_k{spec['k']}_{spec['cond']}"
    elif spec["mesh"] == "hex":
        n = 6
        mesh = cartesian_hexes(n)
        name = f"hex{n}_k{spec['k']}_{spec['cond']}"
    else:
        mesh = make_mesh(spec)
        name = f"quad{spec['n']}_k{spec['k']}_{spec['cond']}"
    data = make_data(spec, mesh.dim)
    k, cond = spec["k"], spec["cond"]
    degrees = list(range(k, -1, -1))
    eta = OS.default_eta(mesh, k)
    t_host = time.perf_counter()
    geo = mesh_geometry(mesh, k, None)
    workers = max(1, min(16, os.cpu_count() or 1))
    chunks = [list(range(i, mesh.n_cells, workers)) for i in range(workers)]
    global _POOL_INPUT
    _POOL_INPUT = (mesh, geo, eta, data)
    # forked workers (run before this process touches the GPU) inherit the inputs
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
        parts = list(ex.map(_oracle_local, chunks))
    _POOL_INPUT = None
    locs = [None] * mesh.n_cells
    for ch, part in zip(chunks, parts):
        for c, L in zip(ch, part):
            locs[c] = L
    t_host = time.perf_counter() - t_host
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    t0 = time.perf_counter()
    cfun = condense_v if cond == "v" else condense_vp
    blocks = [cfun(L) for L in locs]
    lays = [layout(mesh, kl, cond) for kl in degrees]
    S0, b = assemble_condensed(mesh, blocks, mesh.dim, lays[0].nF, lays[0].nP)
    S, idx = [S0], []
    for l in range(len(degrees) - 1):
        ii = coarse_indices(lays[l], lays[l + 1])
        idx.append(ii)
        S.append(S[-1][ii][:, ii].tocsr())
    z = [nullspace(mesh, geo, lay) for lay in lays]
    P = OS.Problem(mesh, geo, k, cond, degrees, eta, locs, blocks, lays, S, b, idx, z)
    t1 = time.perf_counter()
    if coarse == "direct":   # the coarsest level solved exactly (sparse LU of the bordered operator)
        H = OS.hierarchy(P, coarse="direct")
    else:
        H = OS.hierarchy(P, coarse="amg", coarse_rtol=1e-3 if mesh.dim == 3 else 1e-2)
        H.amg_nu = 1        # the library's default: one damped-Jacobi sweep per AMG level
    x, its, hist, conv = OS.solve_fgmres(P, rtol=1e-8, H=H)
    t2 = time.perf_counter()
    dt = t2 - t0
    n0 = S0.shape[0]
    return {"value": n0 / dt / 1e9, "unit": "GDOF/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "cpu_count": os.cpu_count(),
            "sample": (f"{name}: {n0} fine DOFs, FGMRES {its} its to 1e-8 ({'converged' if conv else 'NOT converged'}), "
                       + (f"coarsest level by a sparse LU (SciPy SuperLU) of the bordered operator; "
                          if coarse == "direct" else f"{sum(H.coarse_its)} coarse its; ")
                       + f"timed {dt:.1f} s = condensation/assembly/levels "
                       f"{t1 - t0:.1f} s + smoother/coarse setup and FGMRES {t2 - t1:.1f} s (NumPy/SciPy FP64: "
                       f"dense products on up to {threads} BLAS threads, per-cell loops and sparse products on one); "
                       f"untimed local operators {t_host:.1f} s on {workers} processes"),
            "phases_s": {"condense_assemble_levels": round(t1 - t0, 3), "setup_and_fgmres": round(t2 - t1, 3),
                         "local_operators_untimed": round(t_host, 3)}}


def run_batch(args, record=False):
    """256 independent 2D Stokes problems (Cartesian meshes, side ~ U{16..96},
    k ~ U{1..4}, trig-series force with seed 4000+i, v-cond, homogeneous
    Dirichlet): members of equal degree form one disjoint-union problem with one
    FGMRES process and one set of V-cycle coefficients per member, the coarsest
    levels solved by the sparse direct solve (one pinned pressure and one
    projection per member); the four degree groups run concurrently, one host thread and one HIP
    stream each.  A step = setup + solve of every group.  The V-cycle is FP32 and
    the outer solve FP64; launch shapes come from the library's autotuner
    (untimed).  The groups are timed with eager launches and with every V-cycle
    replayed from a captured HIP graph.  With record=True the result is returned
    (a sub-record of the default run) instead of printed."""
    import threading
    import torch
    import paper_2009_13840_amd as H
    from synth import cartesian_quads, trig_series
    from synth.fields import problem_data
    from synth.batch import batch_spec, shifted, region_fields
    spec = batch_spec()
    groups = {}
    for i, (side, k, seed) in enumerate(spec):
        groups.setdefault(k, []).append((i, side, seed))
    width = 2.0
    precision = "fp32" if record else args.precision
    probs = []
    t0 = time.perf_counter()
    for k, mem in sorted(groups.items()):
        meshes = [shifted(cartesian_quads(side), width * j) for j, (_, side, _) in enumerate(mem)]
        fields = [problem_data(None, trig_series(2, seed), 2) for (_, _, seed) in mem]
        U, fo, co = H.Mesh.union(meshes)
        P = H.Problem(U, k, "v", precision=precision, coarse_rtol=args.coarse_rtol)
        P.set_segments(fo, co)
        P.set_data(*region_fields(fields, 2, width))
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            P.bind("cuda:0")
            P.upload()
            P.setup()
            P.autotune()
        probs.append(dict(k=k, P=P, stream=stream, members=len(mem), cells=U.n_cells))
        print(f"[bench] batch degree {k}: {len(mem)} members, {U.n_cells} cells, {P.level_size(0)} fine DOFs "
              f"({time.perf_counter() - t0:.1f}s)", file=sys.stderr, flush=True)
    host_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    dofs = sum(g["P"].level_size(0) for g in probs)
    cells = sum(g["cells"] for g in probs)

    def run_group(g, out):
        P = g["P"]
        with torch.cuda.stream(g["stream"]):
            P.setup()
            out[g["k"]] = P.solve()[1:]

    def step():
        out = {}
        th = [threading.Thread(target=run_group, args=(g, out)) for g in probs]
        for t in th:
            t.start()
        for t in th:
            t.join()
        return out

    def timed(label):
        for w in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            res = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / args.steps
        per = {}
        worst_rel, max_its, ok_all = 0.0, 0, True
        for g in probs:
            its, hist, rel, ok = res[g["k"]]
            m_its, m_rel = g["P"].batch_results()
            worst_rel = max(worst_rel, float(m_rel.max()))
            max_its = max(max_its, int(m_its.max()))
            ok_all = ok_all and bool(ok) and bool((m_rel <= 1e-8).all())
            per[f"k{g['k']}"] = {"members": g["members"], "fine_dofs": g["P"].level_size(0),
                                 "its_max": int(m_its.max()), "its_mean": round(float(m_its.mean()), 2),
                                 "ok": bool(ok), "phase_ms": {kk: round(v, 2) for kk, v in g["P"].timings().items()}}
        print(f"[bench] batch {label}: {dt * 1e3:.1f} ms/step, its max {max_its}, worst member residual "
              f"{worst_rel:.2e}, converged {ok_all}", file=sys.stderr, flush=True)
        return {"ms_per_step": round(dt * 1e3, 3), "gdof_s": round(dofs / dt / 1e9, 6), "fgmres_its_max": max_its,
                "final_rel_residual_max": worst_rel, "converged": ok_all, "groups": per}

    eager = timed("eager")
    for g in probs:
        g["P"].set_graph(True)
    graph = timed("graph")
    best = graph if graph["converged"] and graph["ms_per_step"] <= eager["ms_per_step"] else eager
    rec = {"workload": "batch256", "problems": len(spec), "cells": cells, "fine_dofs": dofs, "rtol": 1e-8,
           "cond": "v", "precision": precision, "host_set_data_s": round(host_s, 2),
           "eager": eager, "graph": graph, "time_to_1e8_ms": best["ms_per_step"],
           "note": "one disjoint-union problem per degree, each member with its own FGMRES process, V-cycle "
                   "coefficients and coarse GMRES; the four groups on four streams; 'graph': every V-cycle "
                   "replayed from a captured HIP graph (coarse GMRES at most 30 columns, tested on the device)"}
    if record:
        return rec
    out = {
        "metric": METRIC, "value": round(dofs / (best["ms_per_step"] / 1e3) / 1e9, 6), "unit": "GDOF/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": best["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32 V-cycle / f64 outer", "data": "synthetic",
        "config": {"workload": "batch256", "problems": len(spec), "cells": cells, "fine_dofs": dofs, "rtol": 1e-8,
                   "cond": "v"},
        "batch": rec, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def _amg_bytes(kind, L, N, d):
    """Algorithmic bytes of one launch of an AMG kernel class on the level with
    sizes L (rows n, next-level rows nc, entries of A, P, B = A P) and the next
    level N: every matrix entry (8-byte value + 4-byte index) and row pointer
    once, every vector read once and written once."""
    n, nc = L["n"], L["nc"]
    vec = n * d * 8
    if kind == "amg_restrict":   # rc = P^T r - B^T x
        return 2 * (nc + 1) * 4 + 12 * (L["nnz_p"] + L["nnz_b"]) + 2 * vec + n * 8 + nc * d * 8
    if kind == "amg_sweep":      # x_out = x_in + w D^-1 (r - A x_in)
        return (n + 1) * 4 + 12 * L["nnz_a"] + n * 8 + 3 * vec
    if kind == "amg_prolong":    # x_out = x_in + P x_c + w D^-1 (r - A x_in - B x_c)
        return 3 * (n + 1) * 4 + 12 * (L["nnz_a"] + L["nnz_b"] + L["nnz_p"]) + n * 8 + 3 * vec + nc * d * 8
    if kind == "amg_dense":      # x = M r, M explicit n x n
        return n * n * 8 + 2 * vec
    raise ValueError(kind)


FP64_VECTOR_PEAK_TFLOPS = 78.6


def local_flops(mesh, spec):
    """Algorithmic FP64 flops of one device build of the local operators (k_local)
    on the mesh: per cell the orthonormal basis by Gram-Schmidt twice (4 nq N1^2),
    the basis gradients (d nq N1^2), stiffness and cell coupling (2 d nq (N1^2 +
    nT^2)), per face the traces of the basis and its normal derivative (2 nqf
    N1^2), the face basis (4 nqf nF^2), the reconstruction right-hand side and the
    face mass products (2 nqf N1 (nF + nT) + 4 nqf nF N1), the Cholesky factor and
    the two triangular solves (n1^3 / 3 + 2 n1^2 nloc), the consistency term
    (2 n1 nloc^2) and per face the stabilisation (2 nF nloc (N1 - nT) + 2 nF
    nloc^2); the rules are those of the device build (operator degree 2k + 2;
    boxes for the 3D meshes used here)."""
    from math import comb
    d, k = mesh.dim, spec["k"]
    N1, nT, nF = comb(k + 1 + d, d), comb(k + d, d), comb(k + d - 1, d - 1)
    n1 = N1 - 1
    od = 2 * k + 2
    cptr = np.asarray(mesh.cell_ptr)
    nfc = np.diff(cptr)
    if d == 2:
        nq = (nfc - 2) * ((od + 3) // 2) ** 2          # polygon fan (as many vertices as faces)
        nqf = np.full_like(nfc, (od + 2) // 2)
    else:
        nq = np.full_like(nfc, ((od + 2) // 2) ** 3)   # boxes
        nqf = np.full_like(nfc, 2 * ((od + 3) // 2) ** 2)  # quadrilateral faces: two triangles
    nloc = nT + nfc * nF
    f = (4 * nq * N1 ** 2 + d * nq * N1 ** 2 + 2 * d * nq * (N1 ** 2 + nT ** 2)
         + nfc * (2 * nqf * N1 ** 2 + 4 * nqf * nF ** 2 + 2 * nqf * N1 * (nF + nT) + 4 * nqf * nF * N1)
         + n1 ** 3 / 3 + 2 * n1 ** 2 * nloc + 2 * n1 * nloc ** 2
         + nfc * (2 * nF * nloc * (N1 - nT) + 2 * nF * nloc ** 2))
    return float(f.sum())


class ByteModel:
    """Algorithmic bytes per launch of every probed kernel class, by level."""

    def __init__(self, P, mesh, spec, precision):
        self.mesh, self.spec, self.P = mesh, spec, P
        self.k, self.cond = spec["k"], spec["cond"]
        self.degrees = list(range(self.k, -1, -1))
        self.nlev = len(self.degrees)
        low = precision in ("fp32", "bf16")
        self.precision = precision
        # vectors (and smoother factors) and the operator's stored values, per level
        self.elem = [4 if (low and l < self.nlev - 1) else 8 for l in range(self.nlev)]
        self.val = [2 if (precision == "bf16" and l < self.nlev - 1) else self.elem[l] for l in range(self.nlev)]
        self._spmv = {}
        self.amg = []
        try:
            lv0 = P.amg_level_info(0)
            self.amg = [P.amg_level_info(l) for l in range(lv0["levels"])]
        except Exception:
            self.amg = []
        self.direct = {}  # sparse direct coarse solve: per tree height (front entries read, front unknowns)
        try:
            for kind in ("fwd", "bwd"):
                self.direct[kind] = P.direct_info("h" + kind).reshape(-1, 2)
        except Exception:
            self.direct = {}

    def spmv(self, level, elem, val=None):
        key = (level, elem, val)
        if key not in self._spmv:
            self._spmv[key] = spmv_bytes(self.mesh, self.k, self.cond, self.degrees[level], elem, val)
        return self._spmv[key]

    def bytes(self, kind, level):
        d = self.mesh.dim
        if kind == "operator":       # two-slot input form: one more vector read
            b, info = self.spmv(level, self.elem[level], self.val[level])
            return b + info["N"] * self.elem[level]
        if kind == "smoother":
            return precond_bytes(self.mesh, self.degrees[level], self.cond, self.elem[level])
        if kind == "coarse_operator":
            return self.spmv(self.nlev - 1, 8)[0]
        if kind == "outer_operator":
            return self.spmv(0, 8)[0]
        if kind in ("direct_fwd", "direct_bwd"):
            # every front entry the pass reads once (8 bytes), its fronts' vectors:
            # forward gathers b and the children's updates and writes v and u,
            # backward gathers [v1; x2] and writes x1 (about three vectors each)
            ent, unk = self.direct[kind[7:]][level]
            return 8 * int(ent) + 3 * 8 * int(unk)
        L = self.amg[level]
        N = self.amg[level + 1] if level + 1 < len(self.amg) else None
        return _amg_bytes(kind, L, N, d)

    def levels(self, kind):
        if kind in ("operator", "smoother"):
            return range(self.nlev - 1)
        if kind == "coarse_operator":
            return [self.nlev - 1]
        if kind == "outer_operator":
            return [0]
        if kind in ("direct_fwd", "direct_bwd"):
            return range(len(self.direct.get(kind[7:], [])))
        return range(len(self.amg))


def kernel_label(kind, mesh, spec, model, level):
    """Kernel name of a probed class on a level, as rocprofv3 lists it."""
    from math import comb
    d = mesh.dim
    if kind in ("operator", "smoother"):
        k = model.degrees[level]
        form = model.precision if model.elem[level] == 4 else "fp64"
        T = STORAGE_TYPES[form if form in STORAGE_TYPES else "fp64"]
        if kind == "operator":
            return fine_kernel_name(d, k, spec["cond"], form)
        p = comb(k + d - 1, d - 1)
        rows = int(np.diff(np.asarray(mesh.cell_ptr)).max()) * (p if spec["cond"] == "v" else d * p)
        return f"k_precond<{T}, {(rows + 63) // 64}, {d if spec['cond'] == 'v' else 1}>"
    return {"amg_restrict": "k_amg_restrict", "amg_sweep": "k_amg_rows<G>", "amg_prolong": "k_amg_prolong_sweep<G>",
            "amg_dense": "k_amg_dense", "coarse_operator": "k = 0 operator (k_spmv_v0 / k_spmv_vp)",
            "outer_operator": "level-0 operator, one-slot form", "direct_fwd": "k_nd_fwd",
            "direct_bwd": "k_nd_bwd"}[kind]


def probe_table(P, model):
    """Launches, time and algorithmic bytes of every armed class, per level."""
    import paper_2009_13840_amd as H
    out = {}
    for kind, bit in H.PROBE.items():
        rows = []
        for l in model.levels(kind):
            n, ms, alln = P.probe_read(bit, l)
            if n:
                rows.append({"level": l, "launches": n, "ms": ms, "all_launches": alln,
                             "bytes_per_launch": int(model.bytes(kind, l))})
        if rows:
            out[kind] = rows
    return out


def roofline_from(table, kind, label, workload):
    rows = table[kind]
    launches = sum(r["launches"] for r in rows)
    all_launches = sum(r["all_launches"] for r in rows)
    ms = sum(r["ms"] for r in rows)
    nbytes = sum(r["launches"] * r["bytes_per_launch"] for r in rows)
    achieved = nbytes / (ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(workload, label),
            "kernel": label, "class": kind, "timed_launches": launches, "launches": all_launches,
            "avg_launch_ms": round(ms / launches, 5),
            "bytes_per_launch": int(nbytes / launches),
            "levels": [{"level": r["level"], "launches": r["launches"], "avg_us": round(1e3 * r["ms"] / r["launches"], 2),
                        "bytes_per_launch": r["bytes_per_launch"],
                        "frac": round(r["bytes_per_launch"] / (r["ms"] / r["launches"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
                       for r in rows]}


def coarse_label(P, dim, args):
    """What the problem's coarsest-level solver is (the option, or what AUTO chose)."""
    try:
        sizes = P.direct_info("sizes")
        return (f"sparse direct solve (nested dissection, multifrontal elimination on the device: "
                f"{sizes[0]} fronts, {sizes[1]} tree heights, largest front {sizes[4]})")
    except Exception:
        pass
    try:
        P.amg_level_info(0)
        return (f"GMRES to {args.coarse_rtol or (1e-3 if dim == 3 else 1e-2):g} preconditioned by a block-triangular "
                "Stokes preconditioner with a smoothed-aggregation AMG velocity block")
    except Exception:
        return "bordered dense inverse" if args.coarse in ("auto", "dense") else f"coarse_mode {args.coarse}"


def run_mode(mesh, data, spec, workload, precision, args, learned=False, x_ref=None, probe=True, copy="convert",
             graph=False, smoother="schwarz"):
    """One configuration of the solver on the workload: host phase and upload
    (untimed), optional training of the learned smoother (untimed), warmup steps,
    then `args.steps` timed steps (setup + solve to 1e-8), each checked for
    convergence.  With probe=True an untimed step first times every probed kernel
    class; the class with the most time is then the only one armed during the
    timed steps (its launches bracketed by events on the library's stream)."""
    import torch
    import paper_2009_13840_amd as H
    M = H.Mesh(mesh)
    P = H.Problem(M, spec["k"], spec["cond"], precision=precision, coarse_rtol=args.coarse_rtol,
                  learned=1 if learned else 0, vcycle_copy=copy, smoother=smoother, coarse_mode=args.coarse)
    t_host = time.perf_counter()
    P.set_data(*data)
    t_host = time.perf_counter() - t_host
    P.bind("cuda:0")
    P.upload()
    if graph:
        P.set_graph(True)
    torch.cuda.synchronize()
    n0 = P.level_size(0)
    tag = (f"{workload} {precision}{' learned' if learned else ''}{' product copy' if copy == 'product' else ''}"
           f"{' graph' if graph else ''}{' ilu' if smoother == 'ilu' else ''}")
    print(f"[bench] {tag}: host phase {t_host:.2f}s, workspace {P.workspace_size() / 2**30:.2f} GiB, "
          f"fine DOFs {n0}", file=sys.stderr, flush=True)
    learned_info = train_learned(P, n0) if learned else None
    failures = []

    def step(label):
        P.setup()
        x, its, hist, rel, ok = P.solve()
        if not ok or not rel <= 1e-8:
            failures.append(f"{label}: its={its} rel={rel:.3e} converged={ok}")
        return x, its, hist, rel, ok

    if args.autotune and probe:
        P.setup()
        print(f"[bench] {tag} autotuned (operator block, patch threads) per level: {P.autotune().tolist()}",
              file=sys.stderr, flush=True)
    for w in range(args.warmup):
        _, its, _, rel, ok = step(f"warmup {w}")
        print(f"[bench] {tag} warmup {w}: its={its} rel={rel:.2e} ok={ok}", file=sys.stderr, flush=True)
    model = ByteModel(P, mesh, spec, precision)
    table_all, dominant = None, None
    if probe:
        P.probe_arm(sum(H.PROBE.values()))
        step("probe step")
        table_all = probe_table(P, model)
        P.probe_arm(0)
        dominant = max(table_all, key=lambda kk: sum(r["ms"] for r in table_all[kk]))
        # one launch in PROBE_STRIDE of the dominant class is timed during the
        # timed steps (the host's event calls would otherwise slow short launches);
        # a stride that shares a factor with the solver's periodic pattern (two
        # sweeps per coarse iteration, a host read every six) would sample one
        # phase of it, e.g. only the launches right after a host synchronisation
        P.probe_arm(H.PROBE[dominant], args.probe_stride)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for st in range(args.steps):
        x, its, hist, rel, ok = step(f"step {st}")
        results.append((its, rel, ok, P.timings()))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    roof = None
    if probe:
        table_timed = probe_table(P, model)
        P.probe_arm(0)
        top = max(table_all[dominant], key=lambda r: r["ms"])["level"]
        label = kernel_label(dominant, mesh, spec, model, top)
        # Per-launch durations from the step with every launch of every class
        # stamped: they agree with the rocprofv3 trace to a few per cent.  With only
        # the dominant class stamped (the timed steps) its launches read 1-1.5 us
        # longer (the stamped launch's start is taken while the unstamped launch
        # before it still drains), which the sampled record beside it shows.
        roof = roofline_from(table_all, dominant, label, workload)
        samp = roofline_from(table_timed, dominant, label, workload)
        roof["measured_in"] = "untimed step with every launch of every probed class stamped"
        roof["timed_steps_sampled"] = {kk: samp[kk] for kk in ("achieved", "frac", "timed_launches", "launches",
                                                             "avg_launch_ms", "levels")}
    for st, (its, rel, ok, tm) in enumerate(results):
        print(f"[bench] {tag} step {st}: its={its} rel={rel:.2e} ok={ok} "
              f"{json.dumps({kk: round(v, 3) for kk, v in tm.items()})}", file=sys.stderr, flush=True)
    its, rel, ok, tm = results[-1]
    vc_gdofs = n0 * tm["vcycles"] / (tm["vcycle_ms"] / 1e3) / 1e9 if tm["vcycle_ms"] > 0 else None
    rec = {"precision": precision, "learned": learned, "vcycle_copy": copy, "graph": graph, "smoother": smoother,
           "time_to_1e8_ms": round(dt * 1e3, 3),
           "gdof_s": round(n0 / dt / 1e9, 6), "vcycle_gdof_s": round(vc_gdofs, 4) if vc_gdofs else None,
           "fgmres_its": its, "final_rel_residual": rel, "converged": not failures, "failures": failures,
           "phase_ms": {kk: round(v, 3) for kk, v in tm.items()}, "host_set_data_s": round(t_host, 3)}
    if learned_info:
        rec["training"] = learned_info
    if tm.get("local_ms", 0) > 0:
        fl = local_flops(mesh, spec)
        ach = fl / (tm["local_ms"] / 1e3) / 1e12
        rec["roofline_local"] = {
            "kernel": "k_local", "bound": "alu", "achieved": round(ach, 3), "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach / FP64_VECTOR_PEAK_TFLOPS, 4), "flops_per_launch": int(fl),
            "avg_launch_ms": round(tm["local_ms"], 4),
            "note": "one launch per step (the local operators of every cell), timed by the library's events "
                    "around it in the last timed step; the kernel is latency-bound (chains of short LDS loops "
                    "between workgroup barriers), not ALU-bound"}
    # V-cycle roofline: algorithmic bytes of every probed launch of the probe step
    # that belongs to the V-cycle, against the V-cycle time of the last timed step
    if table_all:
        vc_kinds = [kk for kk in table_all if kk != "outer_operator"]
        vc_bytes = sum(r["launches"] * r["bytes_per_launch"] for kk in vc_kinds for r in table_all[kk])
        vc_ms_probed = sum(r["ms"] for kk in vc_kinds for r in table_all[kk])
        rec["vcycle_roofline"] = {
            "bytes_per_vcycle": int(vc_bytes / max(tm["vcycles"], 1)),
            "vcycle_ms": round(tm["vcycle_ms"] / max(tm["vcycles"], 1), 4),
            "achieved": round(vc_bytes / max(tm["vcycles"], 1) / (tm["vcycle_ms"] / max(tm["vcycles"], 1) / 1e3) / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(vc_bytes / (tm["vcycle_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "note": "bytes: the probed kernel classes of one untimed step (operator, smoother, coarse operator, "
                    "AMG or the direct solve's passes) per V-cycle; time: the V-cycle's events of the last timed step; Krylov vector "
                    "traffic is not counted in the bytes",
            "probed_kernel_ms_share": round(vc_ms_probed / tm["vcycle_ms"] / 1.0, 4) if tm["vcycle_ms"] else None,
            "classes": {kk: {"launches": sum(r["launches"] for r in table_all[kk]),
                             "ms": round(sum(r["ms"] for r in table_all[kk]), 3),
                             "gbytes": round(sum(r["launches"] * r["bytes_per_launch"] for r in table_all[kk]) / 1e9, 4)}
                        for kk in table_all}}
    if x_ref is not None:
        rec["err_vs_fp64_reference"] = float(torch.linalg.norm(x - x_ref) / torch.linalg.norm(x_ref))
    return P, x, rec, roof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="voronoi16384_k3_v", choices=sorted(WORKLOADS) + ["batch256"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"],
                    help="precision of the headline run (the other modes are reported beside it)")
    ap.add_argument("--coarse-rtol", type=float, default=0.0,
                    help="coarsest-level GMRES tolerance (0: the library's default, 1e-3 in 3D and 1e-2 in 2D)")
    ap.add_argument("--coarse", default="auto", choices=["auto", "direct", "amg", "gmres", "dense"],
                    help="coarsest-level solver (auto: the sparse direct solve whenever its fronts fit, "
                         "else AMG-preconditioned GMRES)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch of 256 problems in the default run")
    ap.add_argument("--probe-stride", type=int, default=PROBE_STRIDE,
                    help="time one launch in this many of the dominant kernel class during the timed steps")
    ap.add_argument("--modes", default="fp64,fp32,bf16,learned,graph,ilu",
                    help="comma list of the solver forms timed on the workload: fp64, fp32, bf16, learned, graph "
                         "(V-cycle replayed from a HIP graph), ilu (the paper's ILU(0)-GMRES(2) smoother)")
    ap.add_argument("--largest", default="hex32_k3_vp",
                    help="second workload timed in FP64 and FP32 beside the headline ('none' to skip)")
    ap.add_argument("--cpu-sample-cells", type=int, default=4096)
    ap.add_argument("--learned", action="store_true", help="headline run with the learned smoother")
    ap.add_argument("--autotune", action="store_true",
                    help="pick per-level launch shapes with the library's autotuner first (untimed)")
    ap.add_argument("--traffic-calibration", action="store_true",
                    help="run a plain 1 GiB device copy first (reference point for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the sharding across GPUs is a design only)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch256":
        return run_batch(args)

    # the CPU baseline first: its host-phase workers are forked before this
    # process initialises the GPU
    cpu = None
    if not args.no_cpu_baseline:
        try:
            spec0 = WORKLOADS[args.workload]
            direct = args.coarse in ("auto", "direct")
            cpu = cpu_baseline(spec0, args.cpu_sample_cells, coarse="direct" if direct else "amg")
        except Exception as e:  # pragma: no cover
            cpu = {"error": repr(e)}
        print(f"[bench] cpu baseline: {json.dumps(cpu)}", file=sys.stderr, flush=True)

    import torch

    if args.traffic_calibration:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def workload_inputs(name):
        spec = WORKLOADS[name]
        t = time.perf_counter()
        mesh = make_mesh(spec)
        data = make_data(spec, mesh.dim)
        print(f"[bench] workload {name}: {mesh.n_cells} cells, {mesh.n_faces} faces "
              f"(mesh {time.perf_counter() - t:.1f}s)", file=sys.stderr, flush=True)
        return spec, mesh, data

    spec, mesh, data = workload_inputs(args.workload)
    modes = [m for m in args.modes.split(",") if m]
    head_mode = "learned" if args.learned else args.precision
    if head_mode not in modes:
        modes.insert(0, head_mode)
    # headline first, so the reference solution comes from it when it is FP64
    modes.sort(key=lambda m: (m != head_mode, m != "fp64"))
    records, head = {}, None
    x_ref = None
    for m in modes:
        prec = "fp64" if m in ("fp64", "learned", "graph", "ilu") else m
        P, x, rec, roof = run_mode(mesh, data, spec, args.workload, prec, args, learned=(m == "learned"),
                                   x_ref=x_ref, probe=(m == head_mode), graph=(m == "graph"),
                                   smoother="ilu" if m == "ilu" else "schwarz")
        if x_ref is None:
            # FP64 reference for the error of every form: this problem solved again to 1e-12 (untimed)
            P.set_tolerances(1e-12, 1000, args.coarse_rtol or (1e-3 if mesh.dim == 3 else 1e-2), 300)
            P.setup()
            x_ref, its_ref, _, rel_ref, ok_ref = P.solve()
            x_ref = x_ref.clone()
            rec["err_vs_fp64_reference"] = float(torch.linalg.norm(x - x_ref) / torch.linalg.norm(x_ref))
            ref_info = {"rtol": 1e-12, "fgmres_its": its_ref, "final_rel_residual": rel_ref, "converged": ok_ref,
                        "from": m}
        if m == head_mode:
            head = (P, x, rec, roof)
        else:
            del P
        records[m] = rec
        torch.cuda.synchronize()
    P, x, rec, roof = head
    n0 = P.level_size(0)
    coarse_desc = coarse_label(P, mesh.dim, args)
    # back-substitution of the cell unknowns from the headline solution (outside the step)
    rec_ms = []
    for _ in range(3):
        t1 = time.perf_counter()
        P.recover_cells(x)
        rec_ms.append((time.perf_counter() - t1) * 1e3)
    base = records.get("fp64")
    for m, r in records.items():
        if base and m != "fp64" and r["converged"] and base["converged"]:
            r["speedup_vs_fp64"] = round(base["time_to_1e8_ms"] / r["time_to_1e8_ms"], 4)
            if r.get("vcycle_gdof_s") and base.get("vcycle_gdof_s"):
                r["vcycle_speedup_vs_fp64"] = round(r["vcycle_gdof_s"] / base["vcycle_gdof_s"], 4)
    del P, head
    torch.cuda.empty_cache()

    largest = None
    if args.largest and args.largest != "none" and args.largest != args.workload:
        lspec, lmesh, ldata = workload_inputs(args.largest)
        largest = {"workload": args.largest, "cells": lmesh.n_cells, "faces": lmesh.n_faces, "k": lspec["k"],
                   "cond": lspec["cond"]}
        lref = None
        for form in ("fp64", "fp32", "bf16", "bf16_product"):
            prec = form.split("_")[0]
            LP, lx, lrec, lroof = run_mode(lmesh, ldata, lspec, args.largest, prec, args, x_ref=lref, probe=True,
                                           copy="product" if form.endswith("product") else "convert")
            if form == "fp64":
                lref = lx.clone()
                largest["fine_dofs"] = LP.level_size(0)
                largest["coarse"] = coarse_label(LP, lmesh.dim, args)
                largest["roofline"] = lroof
            lrec["err_vs_fp64_reference"] = float(torch.linalg.norm(lx - lref) / torch.linalg.norm(lref))
            largest[form] = lrec
            del LP, lx
            torch.cuda.empty_cache()
        for prec in ("fp32", "bf16", "bf16_product"):
            if largest["fp64"]["converged"] and largest[prec]["converged"]:
                largest[prec]["speedup_vs_fp64"] = round(largest["fp64"]["time_to_1e8_ms"] /
                                                         largest[prec]["time_to_1e8_ms"], 4)
                if largest[prec].get("vcycle_gdof_s") and largest["fp64"].get("vcycle_gdof_s"):
                    largest[prec]["vcycle_speedup_vs_fp64"] = round(largest[prec]["vcycle_gdof_s"] /
                                                                    largest["fp64"]["vcycle_gdof_s"], 4)
        largest["note"] = ("err_vs_fp64_reference: relative difference from the FP64 solution of the same problem "
                           "(both to 1e-8)")

    batch = None
    if not args.no_batch:
        batch = run_batch(args, record=True)
        torch.cuda.empty_cache()

    converged = rec["converged"]
    out = {
        "metric": METRIC,
        "value": round(n0 / (rec["time_to_1e8_ms"] / 1e3) / 1e9, 6) if converged else None,
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["time_to_1e8_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ({"fp64": "f64", "fp32": "f32 V-cycle / f64 outer", "bf16": "bf16-stored f32 V-cycle / f64 outer"}[rec["precision"]]) +
                 (" + bf16 MLP" if rec["learned"] else ""),
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": mesh.n_cells, "faces": mesh.n_faces, "k": spec["k"],
                   "cond": spec["cond"], "levels": list(range(spec["k"], -1, -1)), "fine_dofs": n0,
                   "rtol": 1e-8,
                   "coarse": coarse_desc,
                   "smoother": "GMRES(2), right-preconditioned by cell-patch additive Schwarz"},
        "converged": converged,
        "failures": rec["failures"],
        "time_to_1e8_ms": rec["time_to_1e8_ms"],
        "fgmres_its": rec["fgmres_its"],
        "final_rel_residual": rec["final_rel_residual"],
        "vcycle_gdof_s": rec["vcycle_gdof_s"],
        "phase_ms": rec["phase_ms"],
        "modes": records,
        "fp64_reference": ref_info,
        "host_set_data_s": rec["host_set_data_s"],
        "recover_cells_ms": round(min(rec_ms), 3),
        "roofline": roof,
        "roofline_vcycle": rec.get("vcycle_roofline"),
        "roofline_local": rec.get("roofline_local"),
        "largest_single_gpu": largest,
        "batch256": batch,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if not converged:
        sys.exit(1)


if __name__ == "__main__":
    main()
