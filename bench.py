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


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("k_spmv.hip", "k_solve.hip", "device.h", "dev_common.h"):
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


def spmv_bytes(mesh, k, cond, level_k, dtype_bytes=8):
    """Algorithmic bytes of one application of the level operator: every stored
    value once, the int32 block structure, x read once and y written once."""
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
    return vals * dtype_bytes + idx + 2 * N * dtype_bytes, dict(nnzb=nnzb, N=N, values=vals)


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


def fine_kernel_name(d, k, cond, precision):
    """Name of the fine-level operator kernel in its V-cycle (two-slot input) form."""
    from math import comb
    T = "float" if precision == "fp32" else "double"
    p = comb(k + d - 1, d - 1)
    if cond == "v":
        return f"k_spmv_v<{T}, {d}, {p}, {comb(k + d, d)}, true, 0>"
    return f"k_spmv_vp<{T}, {d * p}, true, 0>"


def train_learned(P, n0, forcings=8, cycles=3, steps=1500, batch=2048, lr=1e-3):
    """Untimed: V-cycle training pairs from seeded discrete forcings b = S x_true
    (x_true ~ N(0, 1) per unknown, seeds 1000+i), He-uniform first layer and
    zero output layer, Adam training on the GPU by the library's kernels."""
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
        xt = torch.from_numpy(np.random.default_rng(1000 + i).standard_normal(n0)).cuda()
        X, T = P.learned_collect(xt, cycles)
        Xs.append(X)
        Ts.append(T)
    X, T = torch.cat(Xs), torch.cat(Ts)
    base = float(0.5 * (T.double() ** 2).sum(dim=1).mean())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = P.learned_train(X, T, steps=steps, batch=batch, lr=lr, seed=7)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    P.setup()
    _, its_plain, _, _, _ = P.solve()
    P.learned_enable(True)
    print(f"[bench] learned smoother: {X.shape[0]} pairs ({t1 - t0:.1f}s), {steps} Adam steps ({t2 - t1:.1f}s), "
          f"loss {hist[:10].mean():.3e} -> {hist[-50:].mean():.3e} (zero predictor {base:.3e})",
          file=sys.stderr, flush=True)
    return {"pairs": int(X.shape[0]), "forcings": forcings, "collect_s": round(t1 - t0, 2),
            "train_steps": steps, "batch": batch, "train_s": round(t2 - t1, 2),
            "loss_first": float(hist[:10].mean()), "loss_last": float(hist[-50:].mean()),
            "loss_zero_predictor": base, "fgmres_its_plain": its_plain}


def cpu_baseline(spec, sample_cells=1024):
    """The oracle as it stands, end to end (local operators, condensation,
    assembly, levels, Schwarz setup, FGMRES to 1e-8), on a smaller mesh of the
    same family; reported in the metric's unit (fine DOFs solved per second)."""
    from threadpoolctl import threadpool_limits
    import oracle.solve as OS
    from synth import voronoi_lloyd, cartesian_quads, cartesian_hexes
    if spec["mesh"] == "voronoi":
        mesh = voronoi_lloyd(sample_cells, spec["seed"])
        name = f"voronoi{sample_cells}_k{spec['k']}_{spec['cond']}"
    elif spec["mesh"] == "hex":
        mesh = cartesian_hexes(4)
        name = f"hex4_k{spec['k']}_{spec['cond']}"
    else:
        mesh = cartesian_quads(spec["n"])
        name = f"quad{spec['n']}_k{spec['k']}_{spec['cond']}"
    data = make_data(spec, mesh.dim)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        P = OS.build(mesh, spec["k"], spec["cond"], data)
        x, its, hist, conv = OS.solve_fgmres(P, rtol=1e-8, coarse="gmres", coarse_rtol=1e-3)
        dt = time.perf_counter() - t0
    n0 = P.S[0].shape[0]
    return {"value": n0 / dt / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": f"{name}: {n0} fine DOFs, {its} FGMRES its, {dt:.1f} s single-thread (NumPy/SciPy FP64)"}


def run_batch(args):
    """256 independent 2D Stokes problems (Cartesian meshes, side ~ U{16..96},
    k ~ U{1..4}, trig-series force with seed 4000+i, v-cond, homogeneous
    Dirichlet): members of equal degree form one disjoint-union problem with one
    FGMRES process per member; the four degree groups run concurrently, one host
    thread and one HIP stream each.  A step = setup + solve of every group."""
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
    probs = []
    t0 = time.perf_counter()
    for k, mem in sorted(groups.items()):
        meshes = [shifted(cartesian_quads(side), width * j) for j, (_, side, _) in enumerate(mem)]
        fields = [problem_data(None, trig_series(2, seed), 2) for (_, _, seed) in mem]
        U, fo, co = H.Mesh.union(meshes)
        P = H.Problem(U, k, "v", precision=args.precision, coarse_rtol=args.coarse_rtol)
        P.set_segments(fo, co)
        P.set_data(*region_fields(fields, 2, width))
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            P.bind("cuda:0")
            P.upload()
        probs.append(dict(k=k, P=P, stream=stream, members=len(mem), cells=U.n_cells))
        print(f"[bench] degree {k}: {len(mem)} members, {U.n_cells} cells, {P.level_size(0)} fine DOFs "
              f"({time.perf_counter() - t0:.1f}s)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dofs = sum(g["P"].level_size(0) for g in probs)
    cells = sum(g["cells"] for g in probs)

    def run_group(g, out):
        P = g["P"]
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

    for w in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    per = {}
    worst_rel, max_its = 0.0, 0
    for g in probs:
        its, hist, rel, ok = res[g["k"]]
        m_its, m_rel = g["P"].batch_results()
        worst_rel = max(worst_rel, float(m_rel.max()))
        max_its = max(max_its, int(m_its.max()))
        per[f"k{g['k']}"] = {"members": g["members"], "fine_dofs": g["P"].level_size(0), "its_max": int(m_its.max()),
                             "its_mean": round(float(m_its.mean()), 2), "ok": bool(ok),
                             "phase_ms": {k: round(v, 2) for k, v in g["P"].timings().items()}}
    out = {
        "metric": METRIC, "value": round(dofs / dt / 1e9, 6), "unit": "GDOF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 V-cycle / f64 outer", "data": "synthetic",
        "config": {"workload": "batch256", "problems": len(spec), "cells": cells, "fine_dofs": dofs, "rtol": 1e-8,
                   "cond": "v", "groups": per},
        "time_to_1e8_ms": round(dt * 1e3, 3), "fgmres_its_max": max_its, "final_rel_residual_max": worst_rel,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="voronoi16384_k3_v", choices=sorted(WORKLOADS) + ["batch256"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--coarse-rtol", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--learned", action="store_true",
                    help="train the learned fine-level smoother first (untimed) and solve with it")
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

    import torch
    import paper_2009_13840_amd as H

    spec = WORKLOADS[args.workload]
    t_mesh = time.perf_counter()
    mesh = make_mesh(spec)
    data = make_data(spec, mesh.dim)
    t_mesh = time.perf_counter() - t_mesh
    print(f"[bench] workload {args.workload}: {mesh.n_cells} cells, {mesh.n_faces} faces "
          f"(mesh {t_mesh:.1f}s)", file=sys.stderr, flush=True)
    M = H.Mesh(mesh)
    P = H.Problem(M, spec["k"], spec["cond"], precision=args.precision, coarse_rtol=args.coarse_rtol,
                  learned=1 if args.learned else 0)
    t_host = time.perf_counter()
    P.set_data(*data)
    t_host = time.perf_counter() - t_host
    P.bind("cuda:0")
    P.upload()
    torch.cuda.synchronize()
    if args.traffic_calibration:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n0 = P.level_size(0)
    print(f"[bench] host local operators {t_host:.2f}s, workspace {P.workspace_size() / 2**30:.2f} GiB, "
          f"fine DOFs {n0}", file=sys.stderr, flush=True)

    def step():
        P.setup()
        return P.solve()

    tuned = None
    if args.autotune:
        P.setup()
        tuned = P.autotune().tolist()
        print(f"[bench] autotuned (operator block, patch threads) per level: {tuned}", file=sys.stderr, flush=True)
    learned_info = None
    if args.learned:
        learned_info = train_learned(P, n0)

    for w in range(args.warmup):
        _, its, _, rel, ok = step()
        print(f"[bench] warmup {w}: its={its} rel={rel:.2e} ok={ok}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for s in range(args.steps):
        x, its, hist, rel, ok = step()
        results.append((its, rel, ok, P.timings()))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    for s, (its, rel, ok, tm) in enumerate(results):
        print(f"[bench] step {s}: its={its} rel={rel:.2e} ok={ok} {json.dumps({k: round(v, 3) for k, v in tm.items()})}",
              file=sys.stderr, flush=True)
    its, rel, ok, tm = results[-1]
    vc_gdofs = n0 * tm["vcycles"] / (tm["vcycle_ms"] / 1e3) / 1e9 if tm["vcycle_ms"] > 0 else None
    # back-substitution of the cell unknowns from the last solution (outside the
    # step): wall time of the call, which returns after its kernel has finished
    rec_ms = []
    for _ in range(3):
        t1 = time.perf_counter()
        P.recover_cells(x)
        rec_ms.append((time.perf_counter() - t1) * 1e3)

    # roofline of the dominant memory-bound kernel: the fine-level operator application
    kind = 2  # the V-cycle's operator application (two-slot input) on level 0
    avg_ms = P.time_kernel(kind, 0, args.kernel_reps)
    elem = 4 if args.precision == "fp32" else 8
    nbytes, info = spmv_bytes(mesh, spec["k"], spec["cond"], spec["k"], elem)
    nbytes += info["N"] * elem  # second slot of the input face part + combined write of the input
    achieved = nbytes / (avg_ms / 1e3) / 1e9
    kname = fine_kernel_name(mesh.dim, spec["k"], spec["cond"], args.precision)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.workload, kname),
            "kernel": kname, "bytes_per_launch": int(nbytes), "avg_launch_ms": round(avg_ms, 5)}
    # the fine-level patch smoother (FP64), the other bandwidth-bound kernel of the V-cycle
    pc_ms = P.time_kernel(1, 0, args.kernel_reps)
    pc_bytes = precond_bytes(mesh, spec["k"], spec["cond"])
    pc_name = precond_kernel_name(mesh, spec["k"], spec["cond"])
    roof_pc = {"bound": "hbm", "achieved": round(pc_bytes / (pc_ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": round(pc_bytes / (pc_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
               "traffic": measured_traffic(args.workload, pc_name), "kernel": pc_name,
               "bytes_per_launch": int(pc_bytes), "avg_launch_ms": round(pc_ms, 5)}

    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(spec)
        except Exception as e:  # pragma: no cover
            cpu = {"error": repr(e)}

    out = {
        "metric": METRIC,
        "value": round(n0 / dt / 1e9, 6),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f64" if args.precision == "fp64" else "f32 V-cycle / f64 outer") + (" + f32 MLP" if args.learned else ""),
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": mesh.n_cells, "faces": mesh.n_faces, "k": spec["k"],
                   "cond": spec["cond"], "levels": list(range(spec["k"], -1, -1)), "fine_dofs": n0,
                   "rtol": 1e-8, "coarse": "gmres 1e-3" if n0 > 4096 else "dense"},
        "time_to_1e8_ms": round(dt * 1e3, 3),
        "fgmres_its": its,
        "final_rel_residual": rel,
        "vcycle_gdof_s": round(vc_gdofs, 4) if vc_gdofs else None,
        "phase_ms": {k: round(v, 3) for k, v in tm.items()},
        # outside the timed step: host-side local operators (incl. the data
        # callbacks) and symbolic AMG hierarchy, before the upload
        "host_set_data_s": round(t_host, 3),
        "recover_cells_ms": round(min(rec_ms), 3),
        "roofline": roof,
        "roofline_smoother": roof_pc,
        "learned": learned_info,
        "autotune": tuned,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
