#!/usr/bin/env python
"""Benchmark of the vertex-patch multigrid solver on one MI355X.

One step = one complete solve A u = b to a relative residual of 1e-10 (CG from
u = 0, preconditioned by the geometric-multigrid V-cycle whose smoother is the
combined, colorized vertex-patch smoother), on a seeded synthetic right-hand
side that is already resident in HBM.  The default workload is the 3D Q4
Poisson problem on 128^3 cells (513^3 = 135,005,697 nodes), 6 levels, V(2,2),
FP32 V-cycle inside FP64 flexible CG.

Reported value: the smoother's throughput on the finest level, DoFs per
second per sweep (nodes (kN+1)^d divided by the time of one sweep), with the
sweep time measured by the library's HIP events around every finest-level
sweep inside the K timed solves.  The JSON line also carries the solve time,
the plain-FP64 solve time on the same right-hand side, the roofline of the
smoother kernel and the CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "patch_sweep_traffic.json")
TRAFFIC_FILE_F64 = os.path.join(ROOT, "profiles", "patch_sweep_traffic_f64.json")

from paper_2407_02100_amd.traffic_probe import kernel_source_hash  # noqa: E402  (hash of the smoother sources)


def color_counts(dim: int, k: int, n: int, vlo: int = 1, vhi: int | None = None):
    """Per color: (closure nodes of the color's patches, interior nodes written).

    A color's patches sit at vertices v with fixed parity per direction; their
    closures [k(v-1), k(v+1)] tile a contiguous node range per direction and
    their interiors hold (2k-1) nodes per direction each.  [vlo, vhi] limits
    the vertices of the slowest direction (one batch of the batched sweep).
    """
    vhi = n - 1 if vhi is None else vhi
    out = []
    for color in range(2 ** dim):
        clo, inner = 1, 1
        for e in range(dim):
            par = (color >> e) & 1
            lo, hi = (vlo, vhi) if e == dim - 1 else (1, n - 1)
            v0 = lo + ((lo & 1) != par)
            npat = (hi - v0) // 2 + 1 if v0 <= hi else 0
            vlast = v0 + 2 * (npat - 1)
            clo *= (k * (vlast - v0 + 2) + 1) if npat > 0 else 0
            inner *= (2 * k - 1) * npat
        out.append((clo, inner))
    return out


def batches(n: int, batch_layers: int):
    """Vertex ranges [lo, hi] of the batches in the slowest direction (one range: whole colors; the library
    batches only levels with more than 2 batch_layers vertex layers)."""
    if batch_layers <= 0 or n - 1 <= 2 * batch_layers:
        return [(1, n - 1)]
    return [(1 + i * batch_layers, min(n - 1, (i + 1) * batch_layers)) for i in range((n - 2) // batch_layers + 1)]


def sweep_bytes(dim: int, k: int, n: int, word: int, batch_layers: int = 0) -> int:
    """Algorithmic bytes of one sweep: per color (and batch) read the closures of u, read b and write u on
    the interiors; a batched sweep reads the closure planes shared by neighbouring batches twice."""
    return sum((clo + 2 * inner) * word for lo, hi in batches(n, batch_layers)
               for clo, inner in color_counts(dim, k, n, lo, hi))


def traffic_per_launch(path: str, workload: str, batch_layers: int, dtype: str):
    """Measured HBM bytes per launch of the smoother from a committed rocprofv3 summary, or None when the
    summary is missing or was taken with other sources, another workload, batch size or precision."""
    if not os.path.exists(path):
        return None
    tr = json.load(open(path))
    if (tr.get("kernel_source_hash") == kernel_source_hash() and tr.get("workload") == workload
            and tr.get("batch_layers", 0) == batch_layers and tr.get("dtype", "f32") == dtype):
        return tr.get("bytes_per_launch")
    return None


def finest_smoother_kernel(dim: int, k: int, n_cells: int, vcycle: str, coef: str) -> str:
    """The smoother kernel the library's automatic choice (vps_config.patches_per_wave = 0) runs on a level."""
    if coef != "const":
        return "patch_color_kernel"
    if dim == 2:
        return "patch_row2_kernel" if n_cells >= 64 and k >= 2 else "patch_color_kernel"
    if k == 1:
        return "patch_color_kernel"
    if (k == 2 and n_cells >= 32) or (k >= 3 and n_cells >= 64):
        return "patch_row5_kernel" if k == 5 else "patch_row3_kernel"
    if k == 5:
        return "patch_big3_kernel"
    if n_cells >= 32 and not (vcycle == "f32" and k == 4):
        return "patch_pair3_kernel"
    return "patch_wave3_kernel"


def launches_per_sweep(dim: int, n: int, batch_layers: int = 0) -> int:
    return sum(1 for lo, hi in batches(n, batch_layers) for clo, inner in color_counts(dim, 1, n, lo, hi) if inner)


def sweep_bytes_separated(dim: int, k: int, n: int, word: int) -> int:
    """Algorithm 3: per color the global residual (read u and b, write r on all nodes), then the
    local solves (read r and u, write u on the interiors)."""
    nodes = (k * n + 1) ** dim
    return sum((3 * nodes + 3 * inner) * word for _, inner in color_counts(dim, k, n))


# ---------------------------------------------------------------------------
# CPU baseline: the oracle (FP64 NumPy/SciPy: assembled CSR operator, dense
# Cholesky patch solves, eq:colorized one factor per color) timed on the host
# cores, in a child process that touches no GPU.  The headline value is its
# sweep rate on a bounded sample of the 3D Q4 family; beside it, the sweep
# and the multigrid-preconditioned CG solve of the 2D Q2 32^2 workload (whole)
# and of 16^3 samples of the 3D Q4 32^3 and variable-coefficient Q2 64^3
# workloads (their full sizes need tens of GB of CSR matrix and minutes).

def _median3(fn, reps=3):
    ts = []
    out = None
    for _ in range(reps):
        t0 = time.perf_counter()
        out = fn()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2], out


def oracle_child(n_cells: int, degree: int, dim: int, budget_s: float):
    from oracle import assemble, multigrid, smoother
    import vps_inputs as vi
    t0 = time.perf_counter()
    A = assemble.assemble_kron(dim, degree, n_cells)
    P = smoother.Patches(dim, degree, n_cells)
    S = smoother.LocalSolvers(A, P, "shared")
    b = vi.seeded_vector(dim, degree, n_cells, 5)
    u = vi.seeded_vector(dim, degree, n_cells, 105)
    setup = time.perf_counter() - t0
    sweeps, t = 0, 0.0
    while t < budget_s or sweeps < 1:
        t1 = time.perf_counter()
        u = smoother.sweep_colorized(A, b, u, P, S)
        t += time.perf_counter() - t1
        sweeps += 1
    n = (degree * n_cells + 1) ** dim
    out = {"dofs": n, "sweeps": sweeps, "seconds": t, "setup_s": setup, "protocol": {}}
    # sweep and solve per workload (median of 3 each; setup of the hierarchy not timed)
    cases = [("poisson2d_q2_n32", "poisson2d_q2_n32", 2, 2, 32, 4, None),
             ("poisson3d_q4_n32", "sample 3D Q4 16^3, 3 levels", 3, 4, 16, 3, None),
             ("varcoef3d_q2_n64", "sample 3D Q2 16^3, 3 levels, rho = exp(GRF), corr. length 1/8, seed 4", 3, 2, 16, 3,
              4)]
    for name, label, d, k, N, L, rho_seed in cases:
        rho = None if rho_seed is None else vi.rho_cells(N, rho_seed)
        H = multigrid.Hierarchy(d, k, N, L, rho=rho, use_kron=rho is None)
        bb = vi.seeded_vector(d, k, N, 1)
        lev = H.levels[-1]
        lev.solvers  # factor the local solvers outside the timing
        uu = vi.seeded_vector(d, k, N, 2)
        reps = 3 if name == "poisson2d_q2_n32" else 1
        t_sw, _ = _median3(lambda: lev.smooth(bb, uu, 1, reverse=False))
        t_so, (x, it, res) = _median3(lambda: multigrid.pcg(H, bb, 1e-10), reps)
        out["protocol"][name] = {"case": label, "nodes": (k * N + 1) ** d, "sweep_s": t_sw, "solve_s": t_so,
                                 "iterations": it, "rel_residual_true": res,
                                 "timing": "median of 3" if reps == 3 else "sweep median of 3, solve once"}
    print(json.dumps(out))


def cpu_baseline(dim: int, degree: int):
    n_cells = 16 if dim == 3 else 128
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-child", str(n_cells), str(degree), str(dim)]
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    rate = d["dofs"] * d["sweeps"] / d["seconds"]
    cpu = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": rate, "unit": "DoF/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle smoother sweeps (eq:colorized, one factor per color: assembled CSR residual + "
                       f"dense Cholesky patch solves, FP64) on {dim}D Q{degree} with {n_cells}^{dim} cells "
                       f"({d['dofs']} nodes), {d['sweeps']} sweeps in {d['seconds']:.1f} s; one thread "
                       f"(OMP/OpenBLAS/MKL threads = 1; SciPy's CSR product is single-threaded anyway); "
                       f"CPU: {cpu}; host threads available: {len(os.sched_getaffinity(0))}"),
            "protocol": d["protocol"]}


# ---------------------------------------------------------------------------
# Other workloads (outside the timed region): time to 1e-10 of the plain,
# mixed-precision and learned forms on the same GPU.

def _solve(torch, vps, vi, name, vcycle=None, reps=3):
    w = vi.WORKLOADS[name]
    dim, k, N = w["dim"], w["degree"], w["n_cells"]
    b = torch.from_numpy(vi.seeded_vector(dim, k, N, w["rhs_seed"])).to("cuda")
    x = torch.empty_like(b)
    with vps.Context(dim, k, N, w["levels"], w["pre"], w["post"], vcycle_dtype=vcycle or w["vcycle"]) as ctx:
        ctx.solve(b, x, rtol=1e-10, maxit=200)
        infos = [ctx.solve(b, x, rtol=1e-10, maxit=200) for _ in range(reps)]
    t = sorted(i["seconds"] for i in infos)[len(infos) // 2]
    return {"solve_s": t, "iterations": infos[-1]["iterations"],
            "rel_residual_true": max(i["rel_residual_true"] for i in infos)}, x


def _median_ms(torch, fn, reps=5, inner=20):
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(inner):
            fn()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / inner)
    return sorted(times)[len(times) // 2]


def run_sweep_protocol(torch, vps, vi, name="poisson3d_q4_n128"):
    """Finest-level sweeps alone: 3 warm-ups, median of 5 runs of 20 sweeps, both algorithms; t_apply."""
    w = vi.WORKLOADS[name]
    dim, k, N = w["dim"], w["degree"], w["n_cells"]
    tdt = torch.float32 if w["vcycle"] == "f32" else torch.float64
    word = 4 if w["vcycle"] == "f32" else 8
    b = torch.from_numpy(vi.seeded_vector(dim, k, N, w["rhs_seed"])).to("cuda", tdt)
    u = torch.from_numpy(vi.seeded_vector(dim, k, N, 100 + w["rhs_seed"])).to("cuda", tdt)
    n = u.numel()
    out = {"workload": name, "dtype": w["vcycle"]}
    for alg, nbytes in (("combined", sweep_bytes(dim, k, N, word)),
                        ("separated", sweep_bytes_separated(dim, k, N, word))):
        with vps.Context(dim, k, N, 1, vcycle_dtype=w["vcycle"], algorithm=alg) as ctx:
            for _ in range(3):
                ctx.smooth(0, u, b, sweeps=1)
            ms = _median_ms(torch, lambda: ctx.smooth(0, u, b, sweeps=1))
            out[alg] = {"sweep_ms": ms, "dof_per_s": n / (ms * 1e-3), "alg_bytes_per_sweep": nbytes,
                        "alg_gbs": nbytes / (ms * 1e-3) / 1e9}
            if alg == "combined":
                Au = torch.empty_like(u)
                for _ in range(3):
                    ctx.apply(0, u, Au)
                out["apply_ms"] = _median_ms(torch, lambda: ctx.apply(0, u, Au))
    # dispatch-order study: the order in which the workgroups of a color visit its patches
    orders = {0: "lexicographic, one slab per XCD", 1: "lexicographic, round-robin over XCDs",
              2: "Morton curve, one slab per XCD", 3: "4x4x4 tiles, one slab per XCD"}
    bl = w.get("batch_layers", 0) or w.get("slab_layers", 0)
    if bl:
        with vps.Context(dim, k, N, 1, vcycle_dtype=w["vcycle"], batch_layers=bl) as ctx:
            for _ in range(3):
                ctx.smooth(0, u, b, sweeps=1)
            ms = _median_ms(torch, lambda: ctx.smooth(0, u, b, sweeps=1))
        nbytes = sweep_bytes(dim, k, N, word, bl)
        out["combined_batched"] = {"batch_layers": bl, "sweep_ms": ms, "dof_per_s": n / (ms * 1e-3),
                                   "alg_bytes_per_sweep": nbytes, "alg_gbs": nbytes / (ms * 1e-3) / 1e9}
    # (on the one-patch-per-wave kernel, the one that visits patches in any of these orders)
    out["patch_order_sweep_ms"] = {}
    for order, label in orders.items():
        with vps.Context(dim, k, N, 1, vcycle_dtype=w["vcycle"], patch_order=order, patches_per_wave=1) as ctx:
            for _ in range(3):
                ctx.smooth(0, u, b, sweeps=1)
            out["patch_order_sweep_ms"][label] = _median_ms(torch, lambda: ctx.smooth(0, u, b, sweeps=1))
    # batch processing (Algorithm 5): slabs of B vertex layers, all colors of a slab in turn
    out["batch_layers_sweep_ms"] = {}
    for bl in (2, 4, 8, 16, 32):
        with vps.Context(dim, k, N, 1, vcycle_dtype=w["vcycle"], batch_layers=bl) as ctx:
            for _ in range(3):
                ctx.smooth(0, u, b, sweeps=1)
            out["batch_layers_sweep_ms"][str(bl)] = _median_ms(torch, lambda: ctx.smooth(0, u, b, sweeps=1))
    out["sweep_over_apply"] = out["combined"]["sweep_ms"] / out["apply_ms"]
    out["separated_over_combined_time"] = out["separated"]["sweep_ms"] / out["combined"]["sweep_ms"]
    out["separated_over_combined_alg_bytes"] = (out["separated"]["alg_bytes_per_sweep"] /
                                                 out["combined"]["alg_bytes_per_sweep"])
    return out


# The paper's table of multigrid timings (32 CPU cores, FP64, residual reduction 1e-12): smoothing and
# vmult time per application, iterations, solve time; context for the same shapes on one MI355X.
PAPER_TABLE = {
    "paper2d_q3_n2048": {"smoothing_s": 0.197856, "vmult_s": 0.034349, "iterations": 6, "solve_s": 12.0369},
    "paper2d_q5_n2048": {"smoothing_s": 0.387558, "vmult_s": 0.0812562, "iterations": 5, "solve_s": 23.3042},
    "paper3d_q5_n128": {"smoothing_s": 2.37646, "vmult_s": 0.213686, "iterations": 6, "solve_s": 115.17},
}


def run_paper_workloads(torch, vps, vi):
    out = {}
    for name, paper in PAPER_TABLE.items():
        w = vi.WORKLOADS[name]
        dim, k, N = w["dim"], w["degree"], w["n_cells"]
        print(f"[bench] paper shape {name}", file=sys.stderr, flush=True)
        b = torch.from_numpy(vi.seeded_vector(dim, k, N, w["rhs_seed"])).to("cuda")
        u = torch.from_numpy(vi.seeded_vector(dim, k, N, w["u0_seed"])).to("cuda")
        x = torch.empty_like(b)
        Au = torch.empty_like(b)
        with vps.Context(dim, k, N, w["levels"], w["pre"], w["post"], vcycle_dtype=w["vcycle"]) as ctx:
            L = w["levels"] - 1
            ctx.smooth(L, u, b, sweeps=1)
            sweep_ms = _median_ms(torch, lambda: ctx.smooth(L, u, b, sweeps=1), reps=3, inner=3)
            ctx.apply(L, u, Au)
            vmult_ms = _median_ms(torch, lambda: ctx.apply(L, u, Au), reps=3, inner=5)
            ctx.solve(b, x, rtol=1e-12, maxit=100)
            info = ctx.solve(b, x, rtol=1e-12, maxit=100)
        n = b.numel()
        byt = sweep_bytes(dim, k, N, 8, 0)  # algorithmic bytes of one FP64 sweep on whole colors
        out[name] = {"nodes": n, "smoothing_s": sweep_ms * 1e-3, "vmult_s": vmult_ms * 1e-3,
                     "iterations": info["iterations"], "solve_s": info["seconds"],
                     "rel_residual_true": info["rel_residual_true"],
                     "smoother_dof_per_s": n / (sweep_ms * 1e-3),
                     "smoother_kernel": finest_smoother_kernel(dim, k, N, "f64", "const"),
                     "smoother_alg_bytes_per_sweep": byt, "smoother_frac_of_8tbs": byt / (sweep_ms * 1e-3) / 8e12,
                     "paper_cpu_32_cores": paper}
        del b, u, x, Au
    return out


def run_extras(torch, vps, vi):
    out = {}
    out["paper_shapes_fp64"] = run_paper_workloads(torch, vps, vi)
    print("[bench] sweep protocol (combined and separated), finest level", file=sys.stderr, flush=True)
    out["sweep_protocol"] = run_sweep_protocol(torch, vps, vi)
    print("[bench] small workloads", file=sys.stderr, flush=True)
    for name in ("poisson2d_q2_n32", "poisson3d_q4_n32"):
        out[name], _ = _solve(torch, vps, vi, name)
    print("[bench] mixed precision, 3D Q3 64^3", file=sys.stderr, flush=True)
    r64, x64 = _solve(torch, vps, vi, "poisson3d_q3_n64", vcycle="f64")
    r32, x32 = _solve(torch, vps, vi, "poisson3d_q3_n64", vcycle="f32")
    diff = float(torch.linalg.vector_norm(x32 - x64) / torch.linalg.vector_norm(x64))
    out["poisson3d_q3_n64"] = {"plain_f64": r64, "f32_vcycle": r32,
                               "speedup_f32_vs_f64": r64["solve_s"] / r32["solve_s"],
                               "rel_diff_solution_f32_vs_f64": diff}
    print("[bench] learned scaling, 3D Q2 64^3", file=sys.stderr, flush=True)
    from paper_2407_02100_amd import learned
    res = {}
    for tag, cl in (("corr_len_1/8", 1.0 / 8.0), ("corr_len_1/16", 1.0 / 16.0)):
        t0 = time.perf_counter()
        X, T, C, R = learned.training_set([1000, 1001, 1002, 1003], n_cells=64, levels=5, total=200_000,
                                          corr_len=cl)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p, hist = learned.train(X, T, epochs=30)
        cmp = learned.compare(p, n_cells=64, levels=5, rho_seed=4, rhs_seed=4, corr_len=cl)
        for v in cmp.values():
            v.pop("residual_history", None)
        res[tag] = {"targets_and_dataset_s": t1 - t0, "train_s": hist["seconds"], "train_samples": hist["train_samples"],
                    "val_loss_plain": learned.baseline_loss(T[: hist["val_samples"]]),
                    "val_loss_learned": hist["val_loss"][-1], "plain": cmp["mean"], "learned": cmp["learned"],
                    "exact_targets": cmp["exact"], "exact_local_solver": cmp["exact_solver"],
                    "speedup_learned_vs_plain": (cmp["mean"]["seconds"] / cmp["learned"]["seconds"]
                                                 if cmp["mean"]["status"] == 0 else None)}
    out["varcoef3d_q2_n64"] = res
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="poisson3d_q4_n128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64-reference", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (mixed Q3, learned Q2, small problems)")
    ap.add_argument("--oracle-child", nargs=3, type=int, metavar=("N", "K", "D"))
    args = ap.parse_args()

    if args.oracle_child:
        n, k, d = args.oracle_child
        oracle_child(n, k, d, budget_s=8.0)
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the smoother runs on a single MI355X "
              "(sharding across GPUs is not implemented); use --gpus 1", file=sys.stderr)
        return 2

    import vps_inputs as vi
    w = vi.WORKLOADS[args.workload]
    dim, k, N = w["dim"], w["degree"], w["n_cells"]
    if w["coef"] != "const":
        print("bench.py times the constant-coefficient workloads", file=sys.stderr)
        return 2

    # the CPU baseline runs first, before this process touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(dim, k)

    import torch
    from paper_2407_02100_amd import vps

    print(f"[bench] workload {args.workload}: generating the right-hand side", file=sys.stderr, flush=True)
    b_host = vi.seeded_vector(dim, k, N, w["rhs_seed"])
    n = b_host.size
    b = torch.from_numpy(b_host).to("cuda")
    del b_host
    x = torch.empty_like(b)
    word = 4 if w["vcycle"] == "f32" else 8

    # measured copy bandwidth (context for the roofline)
    src = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst

    bl = w.get("batch_layers", 0)
    ctx = vps.Context(dim, k, N, w["levels"], w["pre"], w["post"], vcycle_dtype=w["vcycle"], batch_layers=bl)
    print(f"[bench] warmup {args.warmup} solves", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        ctx.solve(b, x, rtol=1e-10, maxit=100)
    ctx.timing_enable(True)
    print(f"[bench] timing {args.steps} solves", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [ctx.solve(b, x, rtol=1e-10, maxit=100) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tim = ctx.timing_get()
    ctx.timing_enable(False)
    ctx.close()
    ms_per_step = (t1 - t0) / args.steps * 1e3

    L = w["levels"] - 1
    kname = finest_smoother_kernel(dim, k, N, w["vcycle"], w.get("coef", "const"))
    sweeps = tim["smooth_sweeps"][L]
    t_sm = tim["smooth_s"][L]
    value = n * sweeps / t_sm
    # one launch per (batch, color) on the finest level
    lps = launches_per_sweep(dim, N, bl)
    launches = sweeps * lps
    bytes_sweep = sweep_bytes(dim, k, N, word, bl)
    per_launch_s = t_sm / launches
    achieved = bytes_sweep / lps / per_launch_s / 1e9

    traffic = traffic_per_launch(TRAFFIC_FILE, args.workload, bl, w["vcycle"])

    f64 = None
    if not args.no_f64_reference and w["vcycle"] == "f32":
        print("[bench] plain FP64 reference solve", file=sys.stderr, flush=True)
        bl64 = w.get("batch_layers_f64", bl)
        ctx64 = vps.Context(dim, k, N, w["levels"], w["pre"], w["post"], vcycle_dtype="f64", batch_layers=bl64)
        ctx64.solve(b, x, rtol=1e-10, maxit=100)
        ctx64.timing_enable(True)
        i64 = ctx64.solve(b, x, rtol=1e-10, maxit=100)
        t64 = ctx64.timing_get()
        ctx64.close()
        lps64 = launches_per_sweep(dim, N, bl64)
        bytes64 = sweep_bytes(dim, k, N, 8, bl64)
        per64 = t64["smooth_s"][L] / (t64["smooth_sweeps"][L] * lps64)
        ach64 = bytes64 / lps64 / per64 / 1e9
        f64 = {"solve_s": i64["seconds"], "iterations": i64["iterations"],
               "rel_residual_true": i64["rel_residual_true"],
               "smoother_dof_per_s": n * t64["smooth_sweeps"][L] / t64["smooth_s"][L],
               "smoother_gbs": bytes64 * t64["smooth_sweeps"][L] / t64["smooth_s"][L] / 1e9,
               "batch_layers": bl64,
               "roofline": {"bound": "hbm", "achieved": ach64, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": ach64 / HBM_PEAK_GBS,
                            "traffic": traffic_per_launch(TRAFFIC_FILE_F64, args.workload, bl64, "f64"),
                            "kernel": f"{finest_smoother_kernel(dim, k, N, 'f64', w.get('coef', 'const'))} "
                                      "(one color launch of the FP64 smoother, finest level)",
                            "avg_launch_us": per64 * 1e6, "bytes_per_launch": bytes64 / lps64,
                            "launches_per_sweep": lps64}}

    extras = {} if args.no_extras else run_extras(torch, vps, vi)

    solve_s = sum(i["seconds"] for i in infos) / len(infos)
    total_phases = (sum(tim["smooth_s"]) + sum(tim["residual_s"]) + sum(tim["restrict_s"]) +
                    sum(tim["prolong_s"]) + tim["coarse_s"] + tim["cg_operator_s"] + tim["cg_vector_s"])
    out = {
        "metric": "smoother DoF/s, % HBM peak; solve time to 1e-10, plain vs mixed/learned",
        "value": value,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w["vcycle"] == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload,
                   "problem": f"-Laplace(u)=f on [0,1]^{dim}, Q{k}, {N}^{dim} cells, {n} nodes",
                   "levels": w["levels"], "cycle": f"V({w['pre']},{w['post']})",
                   "vcycle_dtype": w["vcycle"], "outer": "FP64 flexible CG" if w["vcycle"] == "f32" else "FP64 PCG",
                   "rtol": 1e-10, "rhs": f"uniform [-1,1] on free nodes, seed {w['rhs_seed']}",
                   "batch_layers": bl,
                   "schedule": "one launch per color; a workgroup per batch of same-color patches"
                               + (f" (a row of {63 // (2 * k)} x-adjacent patches on the finest level)"
                                  if kname == "patch_row3_kernel" else "")},
        "solve": {"seconds": solve_s, "iterations": infos[-1]["iterations"],
                  "rel_residual_true": max(i["rel_residual_true"] for i in infos),
                  "vcycles_timed": tim["vcycles"]},
        "plain_f64": f64,
        "speedup_mixed_vs_f64": (f64["solve_s"] / solve_s) if f64 else None,
        "phase_split": {
            "smooth_finest": t_sm / total_phases,
            "smooth_coarser": (sum(tim["smooth_s"]) - t_sm) / total_phases,
            "residual": sum(tim["residual_s"]) / total_phases,
            "transfer": (sum(tim["restrict_s"]) + sum(tim["prolong_s"])) / total_phases,
            "coarse": tim["coarse_s"] / total_phases,
            "cg_operator": tim["cg_operator_s"] / total_phases,
            "cg_vector": tim["cg_vector_s"] / total_phases,
        },
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"{kname} (one color launch of the smoother, finest level)",
                     "avg_launch_us": per_launch_s * 1e6, "bytes_per_launch": bytes_sweep / lps,
                     "launches_per_sweep": lps,
                     "measured_copy_gbs": copy_gbs},
        "cpu_baseline": cpu,
        "other_workloads": extras,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
