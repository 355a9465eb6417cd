#!/usr/bin/env python3
"""Benchmark of the MBPCG hot path on one MI355X.

Headline workload (the top-level fields of the JSON line): the 3-D 7-point
variable-coefficient diffusion operator on a 128^3 grid (n = 2,097,152,
nnz = 14,581,760), log-normal(sigma = 1) cell coefficients, b ~ N(0, 1),
Jacobi (symmetric diagonal) scaling, tolerance 1e-8, s = 4 -- a synthetic,
seeded stand-in for the paper's sparse SPD matrices.  One step = one
complete solve through the C ABI (scaling, random initial block, the
block-CG loop and the least-squares termination) with A and b already
resident in HBM; the metric is time-to-solution, with the plain
Chronopoulos-Gear CG on the same GPU beside it.

The other configured workloads run in the same invocation and are reported
under "configs", each with its own time-to-solution, CG comparison,
roofline of its dominant kernel and CPU-oracle baseline:

  C1  2-D 5-point Poisson 64^2 (n = 4096), Jacobi, s = 4, tol 1e-8
  C3  dense FP64 SPD A = G G^T / n + 1e-3 I, n = 8192, no preconditioning,
      s in {1, 4, 8, 16, 32}, tol 1e-8, against FP64 CG
  C4  the same construction at n = 16384: FP32 (and BF16) products inside
      the FP64 iterative-refinement loop to 1e-10, s in {8, 16, 32},
      against FP64 CG to 1e-10; every result's error against the oracle's
      FP64 reference solution (tests/golden/dense_mixed_16384.json, matched
      by an input hash)
  C5  512 random-graph Laplacians (avg degree 8) + 1e-2 I, n log-uniform in
      [1e3, 2e5], s in {1, 4, 8}, in one persistent launch, against the same
      systems solved one after another

Roofline "achieved" figures are algorithmic bytes (or flops) per launch
over the kernel's average duration measured with HIP events on the
library's stream inside the timed solves; "traffic" is HBM bytes per launch
from committed rocprofv3 counter runs (profiles/), filled only when those
were taken on the current kernel source.

--workload LEG runs one leg alone and prints it as the JSON line (harder
variants: --shift 1e-5 for the dense legs, --inclusions K [--contrast C]
for diffusion3d).
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
PEAK_TF = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
DEFAULT_S = 4
GOLDEN = os.path.join(ROOT, "tests", "golden")


def pad(s: int) -> int:
    S = 1
    while S < s:
        S *= 2
    return S


def host_cpu() -> dict:
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"model": model, "cores_available": avail}


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2608_07327_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


SPMM_SOURCES = ("k_sparse.hip", "dev_common.hpp")
DENSE_SOURCES = ("k_dense.hip", "dev_common.hpp")
BATCH_SOURCES = ("batch.hip", "dev_common.hpp", "dev_spmm.hpp", "dev_sxs.hpp", "dev_dd.hpp")


def kernel_source_hash() -> str:
    return source_hash(SPMM_SOURCES)


def shape_key(S: int, t: dict) -> str:
    """S,T,SL,V,U,W@workgroups of a tile shape and grid as returned by
    Solver.autotune (the counter record is keyed by both: the traffic of one
    shape depends on the grid, which sets how far apart the tiles in flight
    lie)."""
    slots = t["lanes_per_row"] * t["cols_per_lane"] // S
    return ",".join(str(v) for v in (S, t["tile_rows"], slots, t["cols_per_lane"],
                                     t["loads_in_flight"], t["waves_per_simd"])) + \
        f"@{t['workgroups']}"


def traffic_from_profiles(name: str, key: str, sources=SPMM_SOURCES, any_grid=False):
    """HBM bytes per launch of `key` from the committed counter record
    profiles/<name>, if it was taken on the current source of `sources`;
    else None.  any_grid: `key` is a kernel name and the record's one entry
    for it (on whatever grid it ran) is used."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("kernel_hash") != source_hash(sources):
        return None
    ps = rec.get("per_shape", {})
    if any_grid:
        keys = [k for k in ps if k.split("@")[0] == key]
        ent = ps[keys[0]] if len(keys) == 1 else None
    else:
        ent = ps.get(key)
    return None if ent is None else ent.get("bytes_per_launch")


def projected_oracle(run_k, iters_gpu, budget_s, what, extra_per_iter=0.0):
    """The oracle (one thread) on a bounded sample of a solve: run_k(k) runs
    it capped at k iterations and returns its seconds.  Runs of 1, 3 and
    3 + k iterations fit a fixed cost and a per-iteration time, projected to
    the GPU's iteration count."""
    t1 = run_k(1)
    t3 = run_k(3)
    per = max((t3 - t1) / 2.0, 1e-6)
    k = int(max(0, min(iters_gpu - 3, (budget_s - t1 - t3) / per)))
    if k > 0:
        per = max((run_k(3 + k) - t1) / (2 + k), 1e-6)
    fixed = max(t1 - per, 0.0)
    per_total = per + extra_per_iter
    cpu = host_cpu()
    return {
        "value": round(fixed + per_total * iters_gpu, 3), "unit": "s", "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle on {what}: runs of 1, 3 and {3 + k} iterations; fixed cost "
                   f"{fixed:.2f} s + {per_total:.4f} s/iteration, projected to the GPU's "
                   f"{iters_gpu} iterations"),
        "cpu_model": cpu["model"], "host_cores_available": cpu["cores_available"],
    }


def copy_bandwidth(M, torch, dev):
    """GB/s (read + write) of the library's streaming copy over 1 GiB: the
    HBM rate reachable on the box, beside the roofline fractions."""
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


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def sampled_error(x, rec_x, idx):
    """|x - x_ref| / |x_ref| over the golden file's sampled indices."""
    import numpy as np
    xs = np.asarray(x)[idx]
    xr = np.asarray(rec_x)
    return float(np.linalg.norm(xs - xr) / np.linalg.norm(xr))


def golden(name):
    path = os.path.join(GOLDEN, name)
    return json.load(open(path)) if os.path.exists(path) else None


def timed_runs(fn, steps, warmup, torch):
    """warmup untimed calls, then `steps` timed ones between synchronisations;
    returns (seconds per call, last info)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = None
    for _ in range(steps):
        info = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, info


def check(info, what):
    if info["status"] != 0:
        raise RuntimeError(f"{what}: solve failed: {info}")
    return info


# --------------------------------------------------------------------- sparse
def leg_sparse(args, pois, steps, warmup):
    """C2 (headline) or C1."""
    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_2608_07327_amd import mbpcg as M
    from paper_2608_07327_amd import workloads as W

    cfg = W.CFG_POISSON2D if pois else W.CFG_DIFFUSION3D
    A = W.poisson2d(64) if pois else W.diffusion3d(args.grid, inclusions=args.inclusions,
                                                   contrast=args.contrast)
    b = W.rhs(A.n, cfg)
    s = args.s
    S = pad(s)
    seed = W.uniform_block_seed(cfg, s)
    dev = torch.device("cuda:0")
    solver = M.Solver.from_matrix(A)
    bd = torch.as_tensor(b, device=dev)
    x = torch.empty_like(bd)
    log("sparse", "poisson2d 64^2" if pois else f"diffusion3d {args.grid}^3", "n", A.n, "s", s)

    tuned = {}
    widths = {1, s} | (set() if (args.no_sweep or pois) else {1, 2, 4, 8, 16})
    for sw in sorted(widths):
        tuned[sw] = solver.autotune(sw)

    def mb(**kw):
        return check(solver.solve(bd, x=x, s=s, seed=seed, **kw)[1], "mbpcg")

    def cg(**kw):
        return check(solver.cg_solve(bd, x=x, **kw)[1], "cg")

    # timed region: the headline solves (profile level 2: the production
    # launch sequence, kernel by kernel, with HIP events around the block
    # product only, which time it)
    infos = []
    sec, _ = timed_runs(lambda: infos.append(mb(profile=2)) or infos[-1], steps, warmup, torch)
    infos = infos[warmup:]
    cg_sec, cg_info = timed_runs(lambda: cg(profile=2), steps, 0, torch)
    sec_graph, _ = timed_runs(lambda: mb(), steps, 0, torch)
    cg_sec_graph, _ = timed_runs(lambda: cg(), steps, 0, torch)
    iphase = mb(profile=1)   # every phase timed (outside the timed region)
    mb()   # x of the MBPCG solve for the error against the oracle
    xs = x.cpu().numpy()

    spmm_ms = sum(i["ms_spmm"] for i in infos) / max(1, sum(i["spmm_launches"] for i in infos))
    bytes_alg = 12 * A.nnz + 4 * (A.n + 1) + 16 * A.n * S
    achieved = bytes_alg / (spmm_ms * 1e-3) / 1e9
    traffic = None if pois else traffic_from_profiles("spmm_diffusion3d_128_traffic.json",
                                                      shape_key(S, tuned[s]))
    it = iphase["iterations"]
    phases = [v / max(1, it) for v in iphase["ms_phase"][:5]]

    sweep = None
    if not (args.no_sweep or pois):
        sweep = {}
        for sw in (1, 2, 4, 8, 16):
            inf = check(solver.solve(bd, x=x, s=sw, seed=W.uniform_block_seed(cfg, sw),
                                     profile=2)[1], f"sweep s={sw}")
            ms = inf["ms_spmm"] / max(1, inf["spmm_launches"])
            tr = traffic_from_profiles("spmm_diffusion3d_128_traffic.json",
                                       shape_key(pad(sw), tuned[sw]))
            alg_sw = 12 * A.nnz + 4 * (A.n + 1) + 16 * A.n * pad(sw)
            sweep[str(sw)] = {
                "spmm_shape": shape_key(pad(sw), tuned[sw]),
                "spmm_traffic": tr,
                "spmm_traffic_over_algorithmic": None if tr is None else round(tr / alg_sw, 3),
                "iterations": inf["iterations"],
                "seconds": round(inf["ms_total"] / 1e3, 5),
                "ms_per_iter": round(inf["ms_per_iter"], 4),
                "spmm_ms": round(ms, 5),
                "spmm_GBps": round((12 * A.nnz + 4 * (A.n + 1) + 16 * A.n * pad(sw))
                                   / (ms * 1e-3) / 1e9, 1),
                "rel_res_true": inf["rel_res_true"],
            }

    bj = None
    sizes = [int(v) for v in args.block_jacobi.split(",") if v.strip()] if not pois else []
    if sizes:
        bj = {}
        for bs in sizes:
            pre = dict(precond=M.PRECOND_BLOCK_JACOBI, block_size=bs)
            mb(**pre)
            cg(**pre)
            torch.cuda.synchronize()
            q0 = time.perf_counter()
            ib = mb(**pre)
            torch.cuda.synchronize()
            q1 = time.perf_counter()
            ic = cg(**pre)
            torch.cuda.synchronize()
            q2 = time.perf_counter()
            ip = mb(profile=1, **pre)
            bj[str(bs)] = {
                "seconds_graph_mode": round(q1 - q0, 6), "iterations": ib["iterations"],
                "rel_res_true": ib["rel_res_true"],
                "cg_seconds_graph_mode": round(q2 - q1, 6), "cg_iterations": ic["iterations"],
                "cg_rel_res_true": ic["rel_res_true"],
                "ms_per_iter_phases": dict(zip(["product", "xi", "update", "qr", "dir"],
                                               [round(v / max(1, ip["iterations"]), 4)
                                                for v in ip["ms_phase"][:5]])),
            }

    # error against the oracle's x (stored golden of the same input bytes,
    # or the oracle itself on the small system)
    err = None
    if pois:
        xo, io, _ = O.mbpcg_solve(A, b, s, seed=seed)
        if io["iterations"] == it:
            err = float(np.linalg.norm(xs - xo) / np.linalg.norm(xo))
    elif not args.inclusions and args.grid == 128:
        g = golden("diffusion3d_128.json")
        if g is not None and str(s) in g.get("mbpcg", {}):
            o = g["mbpcg"][str(s)]
            for key, xsk in (("iterations", "x_sample"), ("pairwise_iterations", "pairwise_x_sample"),
                             ("fma_iterations", "fma_x_sample")):
                if o.get(key) == it and xsk in o:
                    err = sampled_error(xs, o[xsk], g["sample_index"])
                    break

    cpu = None
    if not args.no_cpu_baseline:
        if pois:
            t0 = time.perf_counter()
            O.mbpcg_solve(A, b, s, seed=seed)
            c = host_cpu()
            cpu = {"value": round(time.perf_counter() - t0, 4), "unit": "s", "cores": 1,
                   "kind": "oracle", "sample": "the whole oracle solve",
                   "cpu_model": c["model"], "host_cores_available": c["cores_available"]}
        else:
            Mo = O.Matrix(A)
            cpu = projected_oracle(
                lambda k: O.mbpcg_solve(Mo, b, s, seed=seed, max_iter=k)[1]["seconds"],
                it, args.cpu_seconds, f"the same {args.grid}^3 diffusion system, s={s}")

    what = ("poisson2d 64^2 5-point, b~N(0,1), Jacobi scaling, tol 1e-8, MBPCG s=%d" % s
            if pois else
            f"diffusion3d {args.grid}^3 7-point, lognormal(sigma=1) coefficients"
            + (f" with {args.inclusions} 4^3 inclusions x{args.contrast:g}" if args.inclusions
               else "") + f", b~N(0,1), Jacobi scaling, tol 1e-8, MBPCG s={s}")
    out = {
        "workload": what, "n": A.n, "nnz": A.nnz, "s": s,
        "value": round(sec, 6), "unit": "s", "steps": steps, "warmup": warmup,
        "ms_per_step": round(sec * 1e3, 3), "dtype": "f64",
        "iterations": it, "rel_res_true": infos[-1]["rel_res_true"],
        "rel_err_vs_oracle": err,
        "cg_seconds": round(cg_sec, 6), "cg_iterations": cg_info["iterations"],
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
                       f"{tuned[s]['lanes_per_row']} lanes/row, {tuned[s]['cols_per_lane']} "
                       f"cols/lane, {tuned[s]['loads_in_flight']} loads in flight, "
                       f"{tuned[s]['workgroups']} workgroups (autotuned); block product + Gram "
                       "epilogue"),
            "avg_ms": round(spmm_ms, 5),
            "bytes_per_launch": bytes_alg,
        },
        "cpu_baseline": cpu,
        "sweep": sweep,
        "block_jacobi": bj,
    }
    if pois:
        out["roofline"]["note"] = ("working set (~2 MB per iteration) is L2-resident: the solve "
                                   "is launch- and latency-bound, not HBM-bound")
        out["us_per_iter"] = round(infos[-1]["ms_per_iter"] * 1e3, 2)
    solver.close()
    return out


# ---------------------------------------------------------------------- dense
def dense_product_roofline(info, n, S, prec, kernel, traffic=None):
    esz = {"fp64": 8, "fp32": 4, "bf16": 2}[prec]
    pm = max(info["ms_spmm"] / max(1, info["spmm_launches"]), 1e-9)
    bytes_prod = esz * n * n
    flops = 2.0 * n * n * S
    peak = PEAK_TF[prec]
    tf = flops / (pm * 1e-3) / 1e12
    gbs = bytes_prod / (pm * 1e-3) / 1e9
    attainable = min(peak, HBM_PEAK_GBS * 1e9 * flops / bytes_prod / 1e12)
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
            "avg_ms": round(pm, 5), "bytes_per_launch": bytes_prod,
            "mfma_TFLOPs": round(tf, 2), "mfma_peak_TFLOPs": peak,
            "mfma_frac": round(tf / peak, 4), "attainable_TFLOPs": round(attainable, 2),
            "attainable_frac": round(tf / attainable, 4)}


def input_sha(A_host, b):
    h = hashlib.sha256()
    h.update(A_host.tobytes())
    h.update(b.tobytes())
    return h.hexdigest()


def golden_err(o, info, x_host, idx):
    """Sampled error against the golden run (of the three rounding variants)
    that took the same number of iterations, or None."""
    for key, xsk in (("iterations", "x_sample"), ("pairwise_iterations", "pairwise_x_sample"),
                     ("fma_iterations", "fma_x_sample")):
        if o.get(key) == info["iterations"] and xsk in o:
            return sampled_error(x_host, o[xsk], idx)
    return None


def leg_dense(args, steps, warmup):
    """C3: dense FP64, s in {1, 4, 8, 16, 32}, against FP64 CG."""
    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_2608_07327_amd import mbpcg as M
    from paper_2608_07327_amd import workloads as W

    dev = torch.device("cuda:0")
    n = args.n or 8192
    cfg = W.CFG_DENSE
    t0 = time.perf_counter()
    A = W.dense_spd_torch(n, cfg, args.shift, device=dev)
    b = W.rhs(n, cfg)
    bd = torch.as_tensor(b, device=dev)
    x = torch.empty_like(bd)
    solver = M.Solver.from_dense(A)
    An = A.cpu().numpy()
    log("dense n", n, f"inputs {time.perf_counter() - t0:.1f} s")
    g = golden(f"dense_{n}.json") if args.shift == 1e-3 else None
    if g is not None and g.get("input_sha256") != input_sha(An, b):
        g = None
    tol = 1e-8
    nrm_b = float(np.linalg.norm(b))

    def true_res():
        return float(torch.linalg.vector_norm(bd - A @ x)) / nrm_b

    runs = {}
    cg_sec, cg_info = timed_runs(lambda: check(solver.cg_solve(
        bd, x=x, tol=tol, precond=M.PRECOND_NONE, profile=2)[1], "cg"), steps, warmup, torch)
    cg_r = true_res()
    cg_err = golden_err(g["cg"], cg_info, x.cpu().numpy(), g["sample_index"]) \
        if g is not None and "cg" in g else None
    for sw in (1, 4, 8, 16, 32):
        sec, info = timed_runs(lambda: check(solver.solve(
            bd, x=x, s=sw, tol=tol, precond=M.PRECOND_NONE, seed=W.uniform_block_seed(cfg, sw),
            profile=2)[1], f"s={sw}"), steps, warmup, torch)
        r = true_res()
        err = None
        if g is not None and str(sw) in g.get("mbpcg", {}):
            err = golden_err(g["mbpcg"][str(sw)], info, x.cpu().numpy(), g["sample_index"])
        runs[sw] = (sec, info, r, err)
    best = min(runs, key=lambda k: runs[k][0])
    sec, info, r, err = runs[best]
    S = pad(best)
    sweep = {}
    for sw, (sec_k, inf_k, r_k, e_k) in runs.items():
        rl = dense_product_roofline(inf_k, n, pad(sw), "fp64", "")
        sweep[str(sw)] = {"seconds": round(sec_k, 5), "iterations": inf_k["iterations"],
                          "rel_res_true": r_k, "rel_err_vs_oracle": e_k,
                          "product_ms": rl["avg_ms"], "product_GBps": rl["achieved"],
                          "product_TFLOPs": rl["mfma_TFLOPs"]}
    cpu = None
    if not args.no_cpu_baseline:
        Mo = O.Matrix(An.T)   # bitwise symmetric: the transposed view is column-major, no copy
        cpu = projected_oracle(
            lambda k: O.mbpcg_solve(Mo, b, best, tol=tol, jacobi=False,
                                    seed=W.uniform_block_seed(cfg, best), max_iter=k)[1]["seconds"],
            info["iterations"], args.cpu_seconds_dense, f"the same dense n={n} system, s={best}")
        del Mo
    out = {
        "workload": (f"dense SPD A = G G^T/n + {args.shift:g} I (G N(0,1) on the 2^-8 grid), "
                     f"n={n}, b~N(0,1), no precond, tol {tol:g}, FP64, best of s in "
                     "{1,4,8,16,32}"),
        "n": n, "s": best, "value": round(sec, 6), "unit": "s", "steps": steps,
        "warmup": warmup, "dtype": "f64", "iterations": info["iterations"],
        "rel_res_true": r, "rel_err_vs_oracle": err,
        "cg_seconds": round(cg_sec, 6), "cg_iterations": cg_info["iterations"],
        "cg_rel_res_true": cg_r, "cg_rel_err_vs_oracle": cg_err,
        "speedup_vs_cg": round(cg_sec / sec, 4),
        "roofline": dense_product_roofline(
            info, n, S, "fp64",
            f"k_dense_f64 S={S} (v_mfma_f64_16x16x4f64, split over column ranges) + reduce/Gram",
            traffic_from_profiles("dense_8192_traffic.json", f"k_dense_f64<{S}>", DENSE_SOURCES,
                                  any_grid=True) if n == 8192 else None),
        "cpu_baseline": cpu,
        "sweep": sweep,
    }
    solver.close()
    del A, An
    torch.cuda.empty_cache()
    return out


def leg_dense_mixed(args, steps, warmup):
    """C4: FP32 / BF16 products in FP64 iterative refinement to 1e-10."""
    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_2608_07327_amd import mbpcg as M
    from paper_2608_07327_amd import workloads as W

    dev = torch.device("cuda:0")
    n = args.n_mixed or 16384
    cfg = W.CFG_DENSE_MIXED
    t0 = time.perf_counter()
    A = W.dense_spd_torch(n, cfg, args.shift, device=dev)
    b = W.rhs(n, cfg)
    bd = torch.as_tensor(b, device=dev)
    x = torch.empty_like(bd)
    solver = M.Solver.from_dense(A)
    An = A.cpu().numpy()
    log("dense-mixed n", n, f"inputs {time.perf_counter() - t0:.1f} s")
    g = golden(f"dense_mixed_{n}.json") if args.shift == 1e-3 else None
    if g is not None and (g.get("input_sha256") != input_sha(An, b) or "ref" not in g):
        g = None
    tol = 1e-10
    nrm_b = float(np.linalg.norm(b))

    def true_res():
        return float(torch.linalg.vector_norm(bd - A @ x)) / nrm_b

    def err_ref():
        if g is None:
            return None
        return sampled_error(x.cpu().numpy(), g["ref"]["x_sample"], g["sample_index"])

    runs = {}
    cg_sec, cg_info = timed_runs(lambda: solver.cg_solve(
        bd, x=x, tol=tol, precond=M.PRECOND_NONE, profile=2)[1], steps, warmup, torch)
    runs["fp64_cg"] = (cg_sec, cg_info, true_res(), err_ref(), 1, "fp64")
    for prec, name, widths in ((M.FP32_IR, "fp32", (8, 16, 32)), (M.BF16_IR, "bf16", (8,))):
        for sw in widths:
            sec, info = timed_runs(lambda: solver.solve(
                bd, x=x, s=sw, precision=prec, ir_tol=tol, precond=M.PRECOND_NONE,
                seed=W.uniform_block_seed(cfg, sw), profile=2)[1],
                steps if name == "fp32" else 1, warmup if name == "fp32" else 0, torch)
            runs[f"{name}_ir_s{sw}"] = (sec, info, true_res(), err_ref(), sw, name)
    sec, info = timed_runs(lambda: solver.solve(
        bd, x=x, s=16, tol=tol, precond=M.PRECOND_NONE, seed=W.uniform_block_seed(cfg, 16),
        profile=2)[1], steps, warmup, torch)
    runs["fp64_s16"] = (sec, info, true_res(), err_ref(), 16, "fp64")
    fp32 = {k: v for k, v in runs.items() if k.startswith("fp32")}
    ok = {k: v for k, v in fp32.items() if v[1]["status"] == 0}
    pick = min(ok or fp32, key=lambda k: runs[k][0])
    sec, info, r, err, sw, prec = runs[pick]
    S = pad(sw)
    sweep = {}
    for k, (sec_k, inf_k, r_k, e_k, sw_k, prec_k) in runs.items():
        rl = dense_product_roofline(inf_k, n, pad(sw_k), prec_k, "")
        sweep[k] = {"seconds": round(sec_k, 5), "iterations": inf_k["iterations"],
                    "outer_iterations": inf_k["outer_iterations"], "status": inf_k["status"],
                    "rel_res_true": r_k, "rel_err_vs_fp64_oracle": e_k,
                    "product_ms": rl["avg_ms"], "product_GBps": rl["achieved"],
                    "product_TFLOPs": rl["mfma_TFLOPs"]}
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's iterative refinement: inner iterations with FP32-rounded
        # products (per-iteration time from a bounded sample) and one FP64
        # product per outer step
        Mlo = O.Matrix(An.T, lo=O.LO_FP32)   # bitwise symmetric: no column-major copy
        M64 = O.Matrix(An.T)
        t0 = time.perf_counter()
        O.matmul_block(M64, b)
        outer_s = time.perf_counter() - t0
        cpu = projected_oracle(
            lambda k: O.mbpcg_solve(Mlo, b, sw, tol=1e-6, jacobi=False, max_iter=k,
                                    seed=W.uniform_block_seed(cfg, sw))[1]["seconds"],
            info["iterations"], args.cpu_seconds_dense,
            f"the same n={n} system, FP32-rounded inner products, s={sw}")
        cpu["value"] = round(cpu["value"] + outer_s * info["outer_iterations"], 3)
        cpu["sample"] += (f"; plus {info['outer_iterations']} outer FP64 products of "
                          f"{outer_s:.2f} s")
        del Mlo, M64
    out = {
        "workload": (f"dense SPD A = G G^T/n + {args.shift:g} I (G N(0,1) on the 2^-8 grid), "
                     f"n={n}, b~N(0,1), no precond, FP64 iterative refinement to {tol:g} with "
                     "FP32 (and BF16) inner products; best FP32 s in {8,16,32}"),
        "n": n, "s": sw, "value": round(sec, 6), "unit": "s", "steps": steps, "warmup": warmup,
        "dtype": "fp32+f64", "iterations": info["iterations"],
        "outer_iterations": info["outer_iterations"], "rel_res_true": r,
        "rel_err_vs_fp64_oracle": err,
        "fp64_oracle_reference": (None if g is None else
                                  {"s": g["ref_s"], "tol": g["ref_tol"],
                                   "iterations": g["ref"]["iterations"],
                                   "vs_numpy_solve": g["ref"]["vs_numpy_solve"],
                                   "error_measured_on": f"{len(g['sample_index'])} sampled "
                                                        "entries"}),
        "cg_seconds": round(cg_sec, 6), "cg_iterations": cg_info["iterations"],
        "speedup_vs_cg": round(cg_sec / sec, 4),
        "roofline": dense_product_roofline(
            info, n, S, "fp32",
            f"k_dense_f32 S={S} (v_mfma_f32_16x16x4f32 on the tiled FP32 copy) + reduce/Gram",
            traffic_from_profiles("dense_mixed_16384_traffic.json", f"k_dense_f32<{S}>",
                                  DENSE_SOURCES, any_grid=True) if n == 16384 else None),
        "cpu_baseline": cpu,
        "sweep": sweep,
    }
    solver.close()
    del A, An
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------- batch
def batch_hash(systems):
    import numpy as np
    h = hashlib.sha256()
    for y in systems:
        for a in (y.A.rowptr, y.A.colind, y.A.vals, y.b):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(np.int64(y.s).tobytes())
    return h.hexdigest()


def leg_batch(args, steps, warmup):
    """C5: 512 graph Laplacians in one persistent launch."""
    import torch

    from oracle import oracle as O
    from paper_2608_07327_amd import mbpcg as M
    from paper_2608_07327_amd import workloads as W

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    systems = W.graph_laplacian_batch(count=args.count)
    log(f"batch of {len(systems)} generated in {time.perf_counter() - t0:.1f} s")
    items = []
    for y in systems:
        items.append({"n": y.A.n, "rowptr": torch.as_tensor(y.A.rowptr, device=dev),
                      "colind": torch.as_tensor(y.A.colind, device=dev),
                      "vals": torch.as_tensor(y.A.vals, device=dev),
                      "b": torch.as_tensor(y.b, device=dev),
                      "x": torch.empty(y.A.n, dtype=torch.float64, device=dev), "s": y.s})
    seed = 500
    # the systems uploaded once into a batch context (outside the timed
    # region, as A is for the single-system legs), its kernel tuned by timed
    # trials, then solves that replay the captured graph
    t0 = time.perf_counter()
    bt = M.Batch(items)
    upload_s = time.perf_counter() - t0
    tuning = bt.autotune(seed=seed)
    log(f"batch tuned: {tuning}")
    _, pinfo = bt.solve(seed=seed, profile=1)   # phase breakdown (stamped run)
    phases = dict(zip(["product", "xi", "update", "qr", "dir", "termination", "setup", "other"],
                      [round(v, 3) for v in pinfo[0]["ms_phase"]]))
    res = {}

    def run():
        res["st"], res["infos"] = bt.solve(seed=seed)
        return res["infos"][0]

    sec, _ = timed_runs(run, steps, warmup, torch)
    infos = res["infos"]
    one_call, _ = timed_runs(lambda: M.solve_batch(items, seed=seed)[1][0], 1, 0, torch)
    log(f"batched solve {sec:.4f} s")
    t0 = time.perf_counter()
    seq_its = []
    for i, (y, it) in enumerate(zip(systems, items)):
        solver = M.Solver.from_csr(y.A.n, it["rowptr"], it["colind"], it["vals"])
        _, inf = solver.solve(it["b"], s=y.s, seed=seed + i)
        seq_its.append(inf["iterations"])
        solver.close()
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    nnz = sum(y.A.nnz for y in systems)
    n_tot = sum(y.A.n for y in systems)
    # the x of the timed batch against the oracle's stored x (same input bytes)
    g = golden(f"batch_{args.count}.json")
    errs = []
    if g is not None and g.get("input_sha256") == batch_hash(systems):
        for it, info, o in zip(items, infos, g["systems"]):
            e = golden_err(o, info, it["x"].cpu().numpy(), o["sample_index"])
            if e is not None:
                errs.append(e)
    prod_b = upd_b = 0
    for y, inf in zip(systems, infos):
        S_ = pad(y.s)
        k = inf["iterations"]
        prod_b += k * (12 * y.A.nnz + 4 * (y.A.n + 1) + 16 * y.A.n * S_)
        upd_b += k * (8 * 8 * y.A.n * S_ + 8 * y.A.n + 4 * 8 * y.A.n * S_)
    prod_s = phases["product"] * 1e-3
    upd_s = (phases["update"] + phases["dir"]) * 1e-3
    # the whole persistent launch is the kernel: its algorithmic bytes (every
    # system's products and streaming phases over its iterations) over its
    # duration (HIP events around the launch on the library's stream, last
    # timed solve); counted bytes per launch from the committed record
    k_ms = infos[0]["ms_phase"][7]
    job_b = prod_b + upd_b
    traffic = traffic_from_profiles("batch_512_traffic.json", f"k_batch@{tuning['workgroups']}",
                                    BATCH_SOURCES) if len(systems) == 512 else None
    roof = {"bound": "hbm",
            "achieved": round(job_b / (k_ms * 1e-3) / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(job_b / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": (f"k_batch on {tuning['workgroups']} workgroups: the whole persistent solve "
                       "(every phase of every system)"),
            "avg_ms": round(k_ms, 3), "bytes_per_launch": job_b,
            "traffic_over_algorithmic": None if traffic is None else round(traffic / job_b, 3),
            "product_phase_GBps": round(prod_b / prod_s / 1e9, 1) if prod_s > 0 else None,
            "update_phases_GBps": round(upd_b / upd_s / 1e9, 1) if upd_s > 0 else None}
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on every 32nd system, scaled by the work of all systems
        # ((nnz + 14 n) s iterations)
        t_s = w_s = w_all = 0.0
        for i, (y, inf) in enumerate(zip(systems, infos)):
            w = float(y.A.nnz + 14 * y.A.n) * y.s * max(1, inf["iterations"])
            w_all += w
            if i % 32 == 0:
                t_s += O.mbpcg_solve(y.A, y.b, y.s, seed=seed + i)[1]["seconds"]
                w_s += w
        c = host_cpu()
        cpu = {"value": round(t_s * w_all / w_s, 3), "unit": "s", "cores": 1, "kind": "oracle",
               "sample": (f"oracle on {len(range(0, len(systems), 32))} of the {len(systems)} "
                          f"systems (every 32nd): {t_s:.2f} s, scaled by the work of all "
                          "systems ((nnz + 14 n) s iterations)"),
               "cpu_model": c["model"], "host_cores_available": c["cores_available"]}
    bt.close()
    out = {
        "workload": (f"{len(systems)} random-graph Laplacians (avg degree 8) + 1e-2 I, n "
                     "log-uniform in [1e3, 2e5], s in {1,4,8}, Jacobi, tol 1e-8, one persistent "
                     "launch replayed from a batch context (systems resident)"),
        "systems": len(systems), "n_total": n_tot, "nnz_total": nnz,
        "value": round(sec, 6), "unit": "s", "steps": steps, "warmup": warmup, "dtype": "f64",
        "status": res["st"], "converged": sum(1 for i in infos if i["status"] == 0),
        "iterations_max": max(i["iterations"] for i in infos),
        "iterations_sum": sum(i["iterations"] for i in infos),
        "worst_rel_res_true": max(i["rel_res_true"] for i in infos),
        "rel_err_vs_oracle_max": max(errs) if errs else None,
        "systems_compared_with_oracle": len(errs),
        "upload_seconds": round(upload_s, 4),
        "one_call_seconds": round(one_call, 4),
        "tuning": tuning,
        "sequential_seconds": round(seq, 4), "sequential_iterations_sum": sum(seq_its),
        "speedup_vs_sequential": round(seq / sec, 3),
        "ms_phases_profiled_run": phases,
        "roofline": roof, "cpu_baseline": cpu,
    }
    return out


# ----------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="all",
                    choices=("all", "diffusion3d", "poisson2d", "dense", "dense-mixed", "batch"))
    ap.add_argument("--legs", default="C1,C3,C4,C5",
                    help="with --workload all: the configs reported beside the headline")
    ap.add_argument("--s", type=int, default=DEFAULT_S)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--n", type=int, default=0, help="dense order (default 8192)")
    ap.add_argument("--n-mixed", type=int, default=0, help="mixed-precision order (default 16384)")
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
    ap.add_argument("--cpu-seconds-dense", type=float, default=8.0)
    ap.add_argument("--leg-steps", type=int, default=3,
                    help="timed solves per configuration of the nested legs (at most --steps)")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--block-jacobi", default="8,16,32",
                    help="sparse workloads: block sizes of the block-Jacobi leg (MBPCG at --s and "
                         "preconditioned CG, graph mode), '' to skip")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2608_07327_amd import mbpcg as M
    leg_steps = max(1, min(args.steps, args.leg_steps))
    leg_warm = min(args.warmup, 1)
    w = args.workload
    if w in ("all", "diffusion3d", "poisson2d"):
        head = leg_sparse(args, w == "poisson2d", args.steps, args.warmup)
        metric = "time-to-solution at rel.res 1e-8 (MBPCG; plain CG on the same GPU beside it)"
    elif w == "dense":
        head = leg_dense(args, args.steps, args.warmup)
        metric = "time-to-solution at rel.res 1e-8, dense FP64 (plain FP64 CG beside it)"
    elif w == "dense-mixed":
        head = leg_dense_mixed(args, args.steps, args.warmup)
        metric = ("time-to-solution at rel.res 1e-10, mixed-precision iterative refinement "
                  "(plain FP64 CG beside it)")
    else:
        head = leg_batch(args, args.steps, args.warmup)
        metric = ("time-to-solution of the whole batch at rel.res 1e-8 (one persistent launch; "
                  "the same systems one after another beside it)")
    log("headline done")
    configs = None
    if w == "all":
        configs = {}
        for leg in [v.strip() for v in args.legs.split(",") if v.strip()]:
            t0 = time.perf_counter()
            try:
                if leg == "C1":
                    configs[leg] = leg_sparse(args, True, leg_steps, leg_warm)
                elif leg == "C3":
                    configs[leg] = leg_dense(args, leg_steps, leg_warm)
                elif leg == "C4":
                    configs[leg] = leg_dense_mixed(args, leg_steps, leg_warm)
                elif leg == "C5":
                    configs[leg] = leg_batch(args, leg_steps, leg_warm)
            except RuntimeError as e:
                configs[leg] = {"error": str(e)}
            log(leg, f"done in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    out = {
        "metric": metric,
        "value": head["value"], "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(head["value"] * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": head["dtype"], "data": "synthetic",
        "config": {k: head[k] for k in ("workload", "n", "nnz", "s") if k in head},
    }
    for k, v in head.items():
        if k not in ("workload", "n", "nnz", "s", "value", "unit", "steps", "warmup",
                     "ms_per_step", "dtype"):
            out[k] = v
    out["roofline"]["copy_GBps"] = copy_bandwidth(M, torch, dev)
    if configs is not None:
        out["configs"] = configs
    print(json.dumps(out))


if __name__ == "__main__":
    main()
