#!/usr/bin/env python3
"""Benchmark of the MBPCG hot path on one MI355X.

Workload: the 3-D 7-point variable-coefficient diffusion operator on a
128^3 grid (n = 2,097,152, nnz = 14,581,760), log-normal(sigma = 1) cell
coefficients, b ~ N(0, 1), Jacobi (symmetric diagonal) scaling, tolerance
1e-8 -- synthetic, seeded stand-in for the paper's sparse SPD matrices.

One step = one complete solve through the C ABI: scaling, random initial
block, the block-CG loop and the least-squares termination, with A and b
already resident in HBM.  The metric is time-to-solution; the same solve
with the plain Chronopoulos-Gear CG on the same GPU is timed beside it.

The block-product kernel's average duration is measured with HIP events on
the library's stream inside the timed solves (profile mode), and its
algorithmic bytes per launch are 12 nnz + 4 (n + 1) + 16 n S (values and
column indices, row pointers, one read of P and one write of Q, S = padded
block width).

Other workloads (--workload), each printing its own JSON line:
  dense        FP64 SPD A = G G^T / n + 1e-3 I, n = 8192, s in {1,4,8,16,32},
               against FP64 CG on the same GPU
  dense-mixed  the same construction at n = 16384: FP32 and BF16 products
               inside the FP64 iterative-refinement loop to 1e-10, s in
               {8,16,32}, against FP64 CG to 1e-10
  batch        512 random-graph Laplacians (avg degree 8, + 1e-2 I, n
               log-uniform in [1e3, 2e5], s in {1,4,8}) in one persistent
               launch, against the same systems solved one after another
Harder variants: --shift 1e-5 for the dense workloads (CG needs many
iterations relative to n), --inclusions K [--contrast C] for diffusion3d
(K highly conducting 4^3 cubes: a few isolated small eigenvalues).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DEFAULT_S = 4


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("k_sparse.hip", "dev_common.hpp", "dev_spmm.hpp"):
        with open(os.path.join(ROOT, "paper_2608_07327_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def shape_key(S: int, t: dict) -> str:
    """S,T,SL,V,U,W of a tile shape as returned by Solver.autotune."""
    slots = t["lanes_per_row"] * t["cols_per_lane"] // S
    return ",".join(str(v) for v in (S, t["tile_rows"], slots, t["cols_per_lane"],
                                     t["loads_in_flight"], t["waves_per_simd"]))


def traffic_from_profiles(key: str):
    """HBM bytes per launch of the block-product shape `key` from committed
    rocprofv3 counter runs, if they were taken on the current kernel source;
    else None."""
    path = os.path.join(ROOT, "profiles", "spmm_diffusion3d_128_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_hash") != kernel_source_hash():
        return None
    ent = rec.get("per_shape", {}).get(key)
    return None if ent is None else ent.get("bytes_per_launch")


def cpu_baseline(A, b, s, seed, iters_gpu, budget_s, what="128^3 diffusion"):
    """The oracle (single thread) on a bounded sample of the same solve: it is
    run for 1, 3 and 3 + k iterations, the per-iteration time and the fixed
    cost are fitted, and the time-to-solution is projected to the GPU's
    iteration count."""
    from oracle import oracle as O
    M = O.Matrix(A)
    t = {}
    for it in (1, 3):
        _, info, _ = O.mbpcg_solve(M, b, s, seed=seed, max_iter=it)
        t[it] = info["seconds"]
    per = max((t[3] - t[1]) / 2.0, 1e-6)
    k = int(max(0, min(iters_gpu, (budget_s - t[1] - t[3]) / per)))
    if k > 0:
        _, info, _ = O.mbpcg_solve(M, b, s, seed=seed, max_iter=3 + k)
        per = max((info["seconds"] - t[1]) / (2 + k), 1e-6)
    fixed = max(t[1] - per, 0.0)
    return {
        "value": fixed + per * iters_gpu,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle MBPCG on the same {what} system, s={s}: runs of 1, 3 and {3 + k} "
                   f"iterations; fixed cost {fixed:.2f} s + {per:.3f} s/iteration, projected to "
                   f"the GPU's {iters_gpu} iterations"),
    }


def copy_bandwidth(M, torch, dev):
    """GB/s (read + write) of the library's streaming copy over 1 GiB: the
    achievable HBM rate that the roofline fractions can be read against."""
    nb = 1 << 30
    src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    M.stream_copy(dst, src, nb)
    torch.cuda.synchronize()
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        M.stream_copy(dst, src, nb)   # default stream: the events above see it
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return round(2 * nb / (ms * 1e-3) / 1e9, 1)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="diffusion3d",
                    choices=("diffusion3d", "poisson2d", "dense", "dense-mixed", "batch"))
    ap.add_argument("--s", type=int, default=DEFAULT_S)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--n", type=int, default=0, help="dense order (default 8192 / 16384)")
    ap.add_argument("--count", type=int, default=512, help="systems of the batch workload")
    ap.add_argument("--shift", type=float, default=1e-3,
                    help="dense workloads: the shift of G G^T / n + shift I (1e-3 as configured; "
                         "smaller is harder for CG)")
    ap.add_argument("--inclusions", type=int, default=0,
                    help="diffusion3d: that many highly conducting cubic inclusions (a few "
                         "isolated small eigenvalues: harder for CG), 0 as configured")
    ap.add_argument("--contrast", type=float, default=1e4,
                    help="diffusion3d with --inclusions: coefficient factor inside them")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--block-jacobi", default="8,16,32",
                    help="sparse workloads: block sizes of the block-Jacobi leg (MBPCG at --s and "
                         "preconditioned CG, graph mode), '' to skip")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB mbpcg_stream_copy (reference for byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload in ("diffusion3d", "poisson2d"):
        bench_sparse(args)
    elif args.workload == "batch":
        bench_batch(args)
    else:
        bench_dense(args, mixed=args.workload == "dense-mixed")


def bench_sparse(args):
    import numpy as np
    import torch

    from paper_2608_07327_amd import mbpcg as M
    from paper_2608_07327_amd import workloads as W

    pois = args.workload == "poisson2d"
    cfg = W.CFG_POISSON2D if pois else W.CFG_DIFFUSION3D
    A = W.poisson2d(64) if pois else W.diffusion3d(args.grid, inclusions=args.inclusions,
                                                   contrast=args.contrast)
    b = W.rhs(A.n, cfg)
    s = args.s
    S = 1
    while S < s:
        S *= 2
    seed = W.uniform_block_seed(cfg, s)
    dev = torch.device("cuda:0")
    solver = M.Solver.from_matrix(A)
    bd = torch.as_tensor(b, device=dev)
    x = torch.empty_like(bd)

    def run(fn, **kw):
        _, info = fn(bd, x=x, **kw)
        if info["status"] != 0:
            raise RuntimeError(f"solve failed: {info}")
        return info

    if args.copy_calibration:
        nb = 1 << 30
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        M.stream_copy(dst, src, nb)
        torch.cuda.synchronize()
        del src, dst

    tuned = {}
    for sw in sorted({1, s} | (set() if args.no_sweep else {1, 2, 4, 8, 16})):
        tuned[sw] = solver.autotune(sw)

    for _ in range(args.warmup):
        run(solver.solve, s=s, seed=seed, profile=1)
        run(solver.cg_solve, profile=1)

    # timed region: MBPCG solves
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [run(solver.solve, s=s, seed=seed, profile=1) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / args.steps

    # same system with plain CG
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    cg_infos = [run(solver.cg_solve, profile=1) for _ in range(args.steps)]
    torch.cuda.synchronize()
    c1 = time.perf_counter()
    cg_sec = (c1 - c0) / args.steps

    # graph-mode (no per-kernel events) time of the same solve, for reference
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for _ in range(args.steps):
        run(solver.solve, s=s, seed=seed)
    torch.cuda.synchronize()
    sec_graph = (time.perf_counter() - g0) / args.steps
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for _ in range(args.steps):
        run(solver.cg_solve)
    torch.cuda.synchronize()
    cg_sec_graph = (time.perf_counter() - g0) / args.steps

    spmm_ms = sum(i["ms_spmm"] for i in infos) / max(1, sum(i["spmm_launches"] for i in infos))
    bytes_alg = 12 * A.nnz + 4 * (A.n + 1) + 16 * A.n * S
    achieved = bytes_alg / (spmm_ms * 1e-3) / 1e9
    traffic = None if pois else traffic_from_profiles(shape_key(S, tuned[s]))
    it = infos[-1]["iterations"]
    phases = [v / max(1, it) for v in infos[-1]["ms_phase"][:5]]

    sweep = None
    if not args.no_sweep:
        sweep = {}
        for sw in (1, 2, 4, 8, 16):
            inf = run(solver.solve, s=sw, seed=W.uniform_block_seed(cfg, sw),
                      profile=1)
            Sw = 1
            while Sw < sw:
                Sw *= 2
            ms = inf["ms_spmm"] / max(1, inf["spmm_launches"])
            sweep[str(sw)] = {
                "iterations": inf["iterations"],
                "seconds": round(inf["ms_total"] / 1e3, 5),
                "ms_per_iter": round(inf["ms_per_iter"], 4),
                "spmm_ms": round(ms, 5),
                "spmm_GBps": round((12 * A.nnz + 4 * (A.n + 1) + 16 * A.n * Sw) / (ms * 1e-3) / 1e9, 1),
                "rel_res_true": inf["rel_res_true"],
            }

    # block-Jacobi preconditioner (the preconditioned form of the method): the
    # same solve and the preconditioned CG, graph mode, and one profiled solve
    # for the per-iteration phases
    bj = None
    sizes = [int(v) for v in args.block_jacobi.split(",") if v.strip()]
    if sizes:
        bj = {}
        for bs in sizes:
            pre = dict(precond=M.PRECOND_BLOCK_JACOBI, block_size=bs)
            run(solver.solve, s=s, seed=seed, **pre)
            run(solver.cg_solve, **pre)
            torch.cuda.synchronize()
            q0 = time.perf_counter()
            ib = run(solver.solve, s=s, seed=seed, **pre)
            torch.cuda.synchronize()
            q1 = time.perf_counter()
            ic = run(solver.cg_solve, **pre)
            torch.cuda.synchronize()
            q2 = time.perf_counter()
            ip = run(solver.solve, s=s, seed=seed, profile=1, **pre)
            bj[str(bs)] = {
                "seconds_graph_mode": round(q1 - q0, 6), "iterations": ib["iterations"],
                "rel_res_true": ib["rel_res_true"],
                "cg_seconds_graph_mode": round(q2 - q1, 6), "cg_iterations": ic["iterations"],
                "cg_rel_res_true": ic["rel_res_true"],
                "ms_per_iter_phases": dict(zip(["product", "xi", "update", "qr", "dir"],
                                               [round(v / max(1, ip["iterations"]), 4)
                                                for v in ip["ms_phase"][:5]])),
            }

    copy_gbs = copy_bandwidth(M, torch, dev)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(A, b, s, seed, it, args.cpu_seconds, "64^2 Poisson" if pois else
                           f"{args.grid}^3 diffusion"
                           + (f" with {args.inclusions} inclusions" if args.inclusions else ""))

    out = {
        "metric": "time-to-solution at rel.res 1e-8 (MBPCG; plain CG on the same GPU beside it)",
        "value": round(sec, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"poisson2d 64^2 5-point, b~N(0,1), Jacobi scaling, tol 1e-8, MBPCG s={s} "
                         "(L2-resident: latency-bound, no meaningful HBM roofline)") if pois else
                        f"diffusion3d {args.grid}^3 7-point, lognormal(sigma=1) coefficients"
                        + (f" with {args.inclusions} 4^3 inclusions x{args.contrast:g}"
                           if args.inclusions else "")
                        + f", b~N(0,1), Jacobi scaling, tol 1e-8, MBPCG s={s}",
            "n": A.n, "nnz": A.nnz, "s": s,
        },
        "iterations": it,
        "rel_res_true": infos[-1]["rel_res_true"],
        "cg_seconds": round(cg_sec, 6),
        "cg_iterations": cg_infos[-1]["iterations"],
        "speedup_vs_cg": round(cg_sec / sec, 4),
        "seconds_graph_mode": round(sec_graph, 6),
        "cg_seconds_graph_mode": round(cg_sec_graph, 6),
        "speedup_vs_cg_graph_mode": round(cg_sec_graph / sec_graph, 4),
        "ms_per_iter_phases": dict(zip(["product", "xi", "update", "qr", "dir"],
                                       [round(v, 4) for v in phases])),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": (f"k_spmm S={S}: {tuned[s]['tile_rows']} rows/tile, "
                       f"{tuned[s]['lanes_per_row']} lanes/row, {tuned[s]['cols_per_lane']} cols/lane, "
                       f"{tuned[s]['loads_in_flight']} loads in flight, {tuned[s]['workgroups']} "
                       f"workgroups (autotuned); block product + Gram epilogue"),
            "avg_ms": round(spmm_ms, 5),
            "bytes_per_launch": bytes_alg,
            "copy_GBps": copy_gbs,
        },
        "cpu_baseline": cpu,
        "sweep": sweep,
        "block_jacobi": bj,
    }
    solver.close()
    print(json.dumps(out))


def dense_on_device(n, tag, torch, dev, shift):
    """workloads.dense_spd with the n^3 product done on the GPU (input
    generation only; the product is exact, so the bytes equal the CPU
    construction's)."""
    from paper_2608_07327_amd import workloads as W
    a = W.dense_spd_torch(n, tag, shift, device=dev)
    torch.cuda.synchronize()
    return a


def bench_dense(args, mixed):
    import numpy as np
    import torch

    from paper_2608_07327_amd import mbpcg as M
    from paper_2608_07327_amd import workloads as W

    dev = torch.device("cuda:0")
    n = args.n or (16384 if mixed else 8192)
    cfg = W.CFG_DENSE_MIXED if mixed else W.CFG_DENSE
    A = dense_on_device(n, cfg, torch, dev, args.shift)
    bd = torch.as_tensor(W.rhs(n, cfg), device=dev)
    x = torch.empty_like(bd)
    solver = M.Solver.from_dense(A)
    tol = 1e-10 if mixed else 1e-8
    nrm_b = float(torch.linalg.vector_norm(bd))

    def timed(fn, **kw):
        for _ in range(args.warmup):
            fn(bd, x=x, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(args.steps):
            _, info = fn(bd, x=x, **kw)
            infos.append(info)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.steps
        info = infos[-1]
        # FP64 residual of the returned x, recomputed here with torch (reported, not used)
        r = float(torch.linalg.vector_norm(bd - A @ x)) / nrm_b
        return sec, info, r

    cg_sec, cg_info, cg_r = timed(solver.cg_solve, tol=tol, precond=M.PRECOND_NONE, profile=1)
    runs = {}
    if mixed:
        for prec, name in ((M.FP32_IR, "fp32"), (M.BF16_IR, "bf16")):
            for sw in (8, 16, 32):
                sec, info, r = timed(solver.solve, s=sw, precision=prec, ir_tol=tol,
                                     precond=M.PRECOND_NONE, seed=W.uniform_block_seed(cfg, sw),
                                     profile=1)
                runs[f"{name}_s{sw}"] = (sec, info, r, sw, name)
        sec, info, r = timed(solver.solve, s=16, tol=tol, precond=M.PRECOND_NONE,
                             seed=W.uniform_block_seed(cfg, 16), profile=1)
        runs["fp64_s16"] = (sec, info, r, 16, "fp64")
    else:
        for sw in (1, 4, 8, 16, 32):
            sec, info, r = timed(solver.solve, s=sw, tol=tol, precond=M.PRECOND_NONE,
                                 seed=W.uniform_block_seed(cfg, sw), profile=1)
            runs[f"fp64_s{sw}"] = (sec, info, r, sw, "fp64")
    ok = {k: v for k, v in runs.items() if v[1]["status"] == 0 and v[2] < 2 * tol}
    pick = min(ok or runs, key=lambda k: (ok or runs)[k][0])
    sec, info, r, sw, prec = runs[pick]
    S = 1
    while S < sw:
        S *= 2
    esz = {"fp64": 8, "fp32": 4, "bf16": 2}[prec]
    prod_ms = max(info["ms_spmm"] / max(1, info["spmm_launches"]), 1e-9)
    bytes_prod = esz * n * n
    flops_prod = 2.0 * n * n * S
    peak_tf = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}[prec]
    sweep = {}
    for k, (sec_k, inf_k, r_k, sw_k, prec_k) in runs.items():
        pm = max(inf_k["ms_spmm"] / max(1, inf_k["spmm_launches"]), 1e-9)
        Sk = 1
        while Sk < sw_k:
            Sk *= 2
        e = {"fp64": 8, "fp32": 4, "bf16": 2}[prec_k]
        sweep[k] = {"seconds": round(sec_k, 5), "iterations": inf_k["iterations"],
                    "outer_iterations": inf_k["outer_iterations"], "status": inf_k["status"],
                    "rel_res_true": r_k, "product_ms": round(pm, 5),
                    "product_GBps": round(e * n * n / (pm * 1e-3) / 1e9, 1),
                    "product_TFLOPs": round(2.0 * n * n * Sk / (pm * 1e-3) / 1e12, 2)}
    out = {
        "metric": ("time-to-solution at rel.res 1e-10, mixed-precision iterative refinement "
                   "(plain FP64 CG on the same GPU beside it)" if mixed else
                   "time-to-solution at rel.res 1e-8, dense FP64 (plain FP64 CG on the same GPU "
                   "beside it)"),
        "value": round(sec, 6), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": prec if prec != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": f"dense SPD A = G G^T/n + {args.shift:g} I, n={n}, b~N(0,1), "
                               f"no precond, tol {tol:g}, best of {sorted(runs)}: {pick}",
                   "n": n, "s": sw, "shift": args.shift},
        "iterations": info["iterations"], "rel_res_true": r,
        "cg_seconds": round(cg_sec, 6), "cg_iterations": cg_info["iterations"],
        "cg_rel_res_true": cg_r, "speedup_vs_cg": round(cg_sec / sec, 4),
        "roofline": {
            "bound": "hbm", "achieved": round(bytes_prod / (prod_ms * 1e-3) / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(bytes_prod / (prod_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": None, "kernel": f"dense product A P ({prec}, S={S}) + reduce/Gram",
            "avg_ms": round(prod_ms, 5), "bytes_per_launch": bytes_prod,
            "mfma_TFLOPs": round(flops_prod / (prod_ms * 1e-3) / 1e12, 2),
            "mfma_peak_TFLOPs": peak_tf,
            "mfma_frac": round(flops_prod / (prod_ms * 1e-3) / 1e12 / peak_tf, 4),
            # fraction of the attainable roofline min(MFMA peak, HBM peak x intensity)
            "attainable_TFLOPs": round(min(peak_tf, HBM_PEAK_GBS * 1e9 * flops_prod / bytes_prod
                                           / 1e12), 2),
            "attainable_frac": round(flops_prod / (prod_ms * 1e-3) / 1e12
                                     / min(peak_tf, HBM_PEAK_GBS * 1e9 * flops_prod / bytes_prod
                                           / 1e12), 4),
        },
        "cpu_baseline": None,
        "sweep": sweep,
    }
    solver.close()
    print(json.dumps(out))


def bench_batch(args):
    import numpy as np
    import torch

    from paper_2608_07327_amd import mbpcg as M
    from paper_2608_07327_amd import workloads as W

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    systems = W.graph_laplacian_batch(count=args.count)
    print(f"[bench] batch of {len(systems)} generated in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    items = []
    for y in systems:
        items.append({"n": y.A.n, "rowptr": torch.as_tensor(y.A.rowptr, device=dev),
                      "colind": torch.as_tensor(y.A.colind, device=dev),
                      "vals": torch.as_tensor(y.A.vals, device=dev),
                      "b": torch.as_tensor(y.b, device=dev),
                      "x": torch.empty(y.A.n, dtype=torch.float64, device=dev), "s": y.s})
    seed = 500
    _, pinfo = M.solve_batch(items, seed=seed, profile=1)   # phase breakdown (stamped run)
    phases = dict(zip(["product", "xi", "update", "qr", "dir", "termination", "setup", "other"],
                      [round(v, 3) for v in pinfo[0]["ms_phase"]]))
    for _ in range(args.warmup):
        M.solve_batch(items, seed=seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, infos = M.solve_batch(items, seed=seed)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    print(f"[bench] batched solve {sec:.4f} s", file=sys.stderr, flush=True)
    # the same systems one after another through the single-system path
    t0 = time.perf_counter()
    seq_its = []
    for i, (y, it) in enumerate(zip(systems, items)):
        solver = M.Solver.from_csr(y.A.n, it["rowptr"], it["colind"], it["vals"])
        _, inf = solver.solve(it["b"], s=y.s, seed=seed + i)
        seq_its.append(inf["iterations"])
        solver.close()
        if (i + 1) % 64 == 0:
            print(f"[bench] sequential {i + 1}/{len(systems)} {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    nnz = sum(y.A.nnz for y in systems)
    n_tot = sum(y.A.n for y in systems)
    worst = max(i["rel_res_true"] for i in infos)
    # algorithmic bytes of the whole job: per system and iteration the block
    # product (CSR once, P read, Q written) and the streaming updates (update
    # 8 n S + n words, direction 4 n S words); the profiled run's stamped
    # phases give the time they took
    def pad(s_):
        S_ = 1
        while S_ < s_:
            S_ *= 2
        return S_
    prod_b = upd_b = 0
    for y, inf in zip(systems, infos):
        S_ = pad(y.s)
        k = inf["iterations"]
        prod_b += k * (12 * y.A.nnz + 4 * (y.A.n + 1) + 16 * y.A.n * S_)
        upd_b += k * (8 * 8 * y.A.n * S_ + 8 * y.A.n + 4 * 8 * y.A.n * S_)
    prod_s = phases["product"] * 1e-3
    upd_s = (phases["update"] + phases["dir"]) * 1e-3
    roof = {"bound": "hbm",
            "achieved": round(prod_b / prod_s / 1e9, 1) if prod_s > 0 else None,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(prod_b / prod_s / 1e9 / HBM_PEAK_GBS, 4) if prod_s > 0 else None,
            "traffic": None,
            "kernel": "k_batch product phase (all systems' block products, summed over the "
                      "profiled run's stamped phases)",
            "bytes_total": prod_b,
            "update_phases_GBps": round(upd_b / upd_s / 1e9, 1) if upd_s > 0 else None,
            "job_GBps": round((prod_b + upd_b) / sec / 1e9, 1)}
    out = {
        "metric": "time-to-solution of the whole batch at rel.res 1e-8 (one persistent launch; "
                  "the same systems solved one after another beside it)",
        "value": round(sec, 6), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{len(systems)} random-graph Laplacians (avg degree 8) + 1e-2 I, "
                               "n log-uniform in [1e3, 2e5], s in {1,4,8}, Jacobi, tol 1e-8",
                   "systems": len(systems), "n_total": n_tot, "nnz_total": nnz},
        "status": st, "converged": sum(1 for i in infos if i["status"] == 0),
        "iterations_max": max(i["iterations"] for i in infos),
        "iterations_sum": sum(i["iterations"] for i in infos),
        "worst_rel_res_true": worst,
        "sequential_seconds": round(seq, 4), "sequential_iterations_sum": sum(seq_its),
        "speedup_vs_sequential": round(seq / sec, 3),
        "ms_phases_profiled_run": phases,
        "roofline": roof, "cpu_baseline": None,
    }
    print(json.dumps(out))
    if out["converged"] != len(systems):
        sys.exit(1)


if __name__ == "__main__":
    main()
