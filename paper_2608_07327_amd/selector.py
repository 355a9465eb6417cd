"""Choosing the block width: the paper's regression models (Sec. 5) refitted
on MI355X measurements.

Sec. 5 predicts the benefit of MBPCG over CG from the matrix size n, its
nonzero count nnz and the CG solve time t: log10(speedup) linear in log10 n,
log10 nnz and log10 t (three-input model), the iteration ratio linear in
log10 n and log10 t, and log10 of the per-iteration time ratio linear in
log10 n and log10 nnz.  Its coefficients were fitted on a V100 and, as the
paper says, change with hardware and implementation.  This module measures
CG and MBPCG (widths 2, 4, 8, 16) on a family of synthetic SPD systems of
growing size and difficulty on the GPU, fits the same three model forms per
width, stores the fit, and picks a width for a new system (or plain CG when
no width is predicted to win).

    python -m paper_2608_07327_amd.selector --out paper_2608_07327_amd/width_model_mi355x.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
import zlib

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "width_model_mi355x.json")
WIDTHS = (2, 4, 8, 16)


# ------------------------------------------------------------------ family
def family():
    """(name, builder) pairs: 2-D Poisson grids, 3-D diffusion with growing
    coefficient contrast, random-graph Laplacians with shrinking shifts
    (slower CG), dense G G^T / n + shift I with shrinking shifts."""
    from . import workloads as W
    out = []
    for m in (64, 128, 256, 512, 1024):
        out.append((f"poisson2d m={m}", lambda m=m: W.poisson2d(m)))
    for m in (32, 64, 96):
        for sg in (1.0, 2.5):
            out.append((f"diffusion3d m={m} sigma={sg}",
                        lambda m=m, sg=sg: W.diffusion3d(m, sigma=sg,
                                                         tag=(W.CFG_DIFFUSION3D, 90, m, int(10 * sg)))))
    for n in (20000, 200000):
        for sh in (1e-2, 1e-4, 1e-6):
            out.append((f"graph n={n} shift={sh:g}",
                        lambda n=n, sh=sh: W.graph_laplacian(
                            n, 8, sh, W.rng_for((W.CFG_BATCH, 91, n, int(round(-math.log10(sh))))))))
    for n in (2048, 4096):
        for sh in (1e-3, 1e-5):
            out.append((f"dense n={n} shift={sh:g}",
                        lambda n=n, sh=sh: W.dense_spd(n, tag=(W.CFG_DENSE, 92, n), shift=sh)))
    return out


# ------------------------------------------------------------- measurement
def _timed(fn, bd, reps, **kw):
    import torch
    _, info = fn(bd, **kw)              # warm-up (plans, graphs, tuning)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, info = fn(bd, **kw)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, info


def measure(systems=None, widths=WIDTHS, tol=1e-8, max_iter=20000, reps=2, log=sys.stderr):
    """CG and MBPCG time-to-solution (graph mode, A and b resident) for each
    system; returns a list of records."""
    import torch

    from . import mbpcg as M
    from . import workloads as W
    dev = torch.device("cuda:0")
    recs = []
    for name, build in (systems or family()):
        A = build()
        dense = isinstance(A, np.ndarray)
        n = A.shape[0] if dense else A.n
        nnz = int(np.count_nonzero(A)) if dense else int(A.nnz)
        b = W.rng_for((93, zlib.crc32(name.encode()))).standard_normal(n)
        solver = M.Solver.from_matrix(A)
        bd = torch.as_tensor(b, device=dev)
        pc = M.PRECOND_NONE if dense else M.PRECOND_JACOBI
        t_cg, icg = _timed(solver.cg_solve, bd, reps, tol=tol, max_iter=max_iter, precond=pc)
        rec = {"name": name, "n": n, "nnz": nnz, "dense": dense, "cg_seconds": t_cg,
               "cg_iterations": icg["iterations"], "cg_status": icg["status"],
               "cg_rel_res_true": icg["rel_res_true"], "mbpcg": {}}
        for s in widths:
            if not dense:
                solver.autotune(s)
            t, inf = _timed(solver.solve, bd, reps, s=s, tol=tol, max_iter=max_iter, precond=pc,
                            seed=W.uniform_block_seed(94, s))
            rec["mbpcg"][str(s)] = {"seconds": t, "iterations": inf["iterations"],
                                    "status": inf["status"], "rel_res_true": inf["rel_res_true"]}
        solver.close()
        recs.append(rec)
        best = min(rec["mbpcg"].items(), key=lambda kv: kv[1]["seconds"])
        print(f"[selector] {name}: n={n} nnz={nnz} CG {t_cg * 1e3:.2f} ms / {icg['iterations']} it; "
              f"best s={best[0]} {best[1]['seconds'] * 1e3:.2f} ms / {best[1]['iterations']} it",
              file=log, flush=True)
    return recs


# ---------------------------------------------------------------- fitting
def _lstsq(X, y):
    coef, *_ = np.linalg.lstsq(X, y, rcond=None)
    res = y - X @ coef
    ss_res = float(res @ res)
    ss_tot = float(((y - y.mean()) ** 2).sum())
    r2 = 1.0 - ss_res / ss_tot if ss_tot > 0 else 1.0
    m, p = X.shape
    r2_adj = 1.0 - (1.0 - r2) * (m - 1) / (m - p) if m > p else float("nan")
    return coef, r2, r2_adj


def fit(recs, widths=WIDTHS, tol=1e-8):
    """Per width, the three model forms of Sec. 5 by least squares on the
    converged pairs: log10 speedup ~ [1, log10 n, log10 nnz, log10 t],
    iteration ratio ~ [1, log10 n, log10 t], log10 per-iteration time ratio
    ~ [1, log10 n, log10 nnz].  A pair counts as converged when both solves
    report success and their true residuals are below 2 tol."""
    models = {}
    for s in widths:
        rows = []
        for r in recs:
            m = r["mbpcg"].get(str(s))
            if m is None or m["status"] != 0 or r["cg_status"] != 0:
                continue
            if not (m.get("rel_res_true", 0.0) < 2 * tol
                    and r.get("cg_rel_res_true", 0.0) < 2 * tol):
                continue
            if m["iterations"] <= 0 or r["cg_iterations"] <= 0:
                continue
            rows.append((math.log10(r["n"]), math.log10(r["nnz"]), math.log10(r["cg_seconds"]),
                         r["cg_seconds"] / m["seconds"], m["iterations"] / r["cg_iterations"],
                         (m["seconds"] / m["iterations"]) / (r["cg_seconds"] / r["cg_iterations"])))
        if len(rows) < 5:
            continue
        a = np.asarray(rows)
        ln, lz, lt = a[:, 0], a[:, 1], a[:, 2]
        one = np.ones(len(a))
        c_sp, r2_sp, r2a_sp = _lstsq(np.stack([one, ln, lz, lt], 1), np.log10(a[:, 3]))
        c_it, r2_it, r2a_it = _lstsq(np.stack([one, ln, lt], 1), a[:, 4])
        c_pt, r2_pt, r2a_pt = _lstsq(np.stack([one, ln, lz], 1), np.log10(a[:, 5]))
        models[str(s)] = {
            "samples": len(a),
            "log10_speedup": {"const": c_sp[0], "log10_n": c_sp[1], "log10_nnz": c_sp[2],
                              "log10_t": c_sp[3], "r2": r2_sp, "r2_adj": r2a_sp},
            "iteration_ratio": {"const": c_it[0], "log10_n": c_it[1], "log10_t": c_it[2],
                                "r2": r2_it, "r2_adj": r2a_it},
            "log10_time_per_iteration_ratio": {"const": c_pt[0], "log10_n": c_pt[1],
                                               "log10_nnz": c_pt[2], "r2": r2_pt,
                                               "r2_adj": r2a_pt},
            "observed_best_speedup": float(a[:, 3].max()),
        }
    return models


def predict_speedup(model, n, nnz, t_cg):
    m = model["log10_speedup"]
    return 10.0 ** (m["const"] + m["log10_n"] * math.log10(n) + m["log10_nnz"] * math.log10(nnz)
                    + m["log10_t"] * math.log10(t_cg))


def choose_width(n, nnz, t_cg, models=None):
    """The width with the largest predicted speedup over CG, or 1 (plain CG)
    when none is predicted to be faster.  t_cg: CG time-to-solution in
    seconds on this GPU (the model's third input, as in Sec. 5)."""
    if models is None:
        models = load_models()
    best, best_sp = 1, 1.0
    for s, m in models.items():
        sp = predict_speedup(m, n, nnz, t_cg)
        if sp > best_sp:
            best, best_sp = int(s), sp
    return best, best_sp


def load_models(path=MODEL_PATH):
    with open(path) as f:
        return json.load(f)["models"]


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--out", default=MODEL_PATH)
    ap.add_argument("--reps", type=int, default=2)
    args = ap.parse_args()
    recs = measure(reps=args.reps)
    models = fit(recs)
    with open(args.out, "w") as f:
        json.dump({"hardware": "one MI355X", "tol": 1e-8, "timing": "graph mode, A and b resident",
                   "records": recs, "models": models}, f, indent=1)
    for s, m in models.items():
        sp = m["log10_speedup"]
        print(f"s={s}: log10 speedup = {sp['const']:.3f} + {sp['log10_n']:.3f} log n + "
              f"{sp['log10_nnz']:.3f} log nnz + {sp['log10_t']:.3f} log t  (R2 {sp['r2']:.3f}, "
              f"{m['samples']} systems)")


if __name__ == "__main__":
    main()
