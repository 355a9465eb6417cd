"""Write tests/golden/dense_8192.json from the CPU oracle alone.

The dense FP64 workload: A = G G^T / n + 1e-3 I (n = 8192, G iid N(0,1) on
the 2^-8 grid, so the bytes of A do not depend on the BLAS that forms it),
b ~ N(0,1), no preconditioning, tolerance 1e-8.  For each block width s the
oracle's Algorithm 1 runs twice -- sequential and blocked-pairwise
reductions -- and the Chronopoulos-Gear CG once.  Stored: iteration counts,
exit diagnostics, the rounding-order noise floor |x_pairwise - x| / |x|, and
x at 4096 fixed indices, plus a hash of the input bytes.

    python tests/golden/make_dense_golden.py [--n 8192] [--s 1,4,8,16,32] [--jobs 6]

Each (s, summation order) is one job of a process pool; results are written
as they arrive, and widths already in the output are skipped.
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2608_07327_amd import workloads as W  # noqa: E402

TOL = 1e-8
_A = {}


def system(n):
    if n not in _A:
        _A[n] = (W.dense_spd(n, W.CFG_DENSE), W.rhs(n, W.CFG_DENSE))
    return _A[n]


def input_hash(A, b):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(A).tobytes())
    h.update(np.ascontiguousarray(b).tobytes())
    return h.hexdigest()


def sample_index(n, k=4096):
    return np.unique(W.rng_for((99, n)).integers(0, n, k))


def job(task):
    n, kind, s, mode = task
    A, b = system(n)
    idx = sample_index(n)
    O.set_summation(mode)
    t = time.time()
    if kind == "cg":
        x, info, _ = O.cg_cg(A, b, tol=TOL, jacobi=False)
    else:
        x, info, _ = O.mbpcg_solve(A, b, s, tol=TOL, jacobi=False,
                                   seed=W.uniform_block_seed(W.CFG_DENSE, s))
    info["seconds_wall"] = time.time() - t
    return task, info, x[idx].tolist(), float(np.linalg.norm(x)), x


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--s", default="1,4,8,16,32")
    ap.add_argument("--jobs", type=int, default=6)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    out = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                   f"dense_{args.n}.json")
    A, b = system(args.n)
    rec = json.load(open(out)) if os.path.exists(out) else {}
    rec.update({"n": args.n, "shift": 1e-3, "tol": TOL, "input_sha256": input_hash(A, b),
                "sample_index": sample_index(args.n).tolist()})
    rec.setdefault("mbpcg", {})
    tasks = []
    if "cg" not in rec:
        tasks.append((args.n, "cg", 1, 0))
    for s in [int(v) for v in args.s.split(",")]:
        if str(s) not in rec["mbpcg"]:
            tasks += [(args.n, "mbpcg", s, 0), (args.n, "mbpcg", s, 1)]
    # longest jobs first
    tasks.sort(key=lambda t: -t[2])
    partial = {}
    with mp.get_context("fork").Pool(args.jobs) as pool:
        for (n, kind, s, mode), info, xs, xn, x in pool.imap_unordered(job, tasks):
            print(kind, s, "pairwise" if mode else "sequential", info["iterations"],
                  f"{info['seconds_wall']:.0f} s", flush=True)
            if kind == "cg":
                rec["cg"] = {"iterations": info["iterations"], "status": info["status"],
                             "rel_res_true": info["rel_res_true"],
                             "seconds": info["seconds"], "x_sample": xs, "x_norm": xn}
            else:
                partial.setdefault(s, {})[mode] = (info, xs, xn, x)
                if len(partial[s]) == 2:
                    i0, xs0, xn0, x0 = partial[s][0]
                    i1, _, _, x1 = partial[s][1]
                    rec["mbpcg"][str(s)] = {
                        "seed": W.uniform_block_seed(W.CFG_DENSE, s),
                        "iterations": i0["iterations"], "status": i0["status"],
                        "best_column": i0["best_column"], "final_width": i0["final_width"],
                        "deflations": i0["deflations"], "used_fallback": i0["used_fallback"],
                        "rel_res_best": i0["rel_res_best"], "rel_res_ls": i0["rel_res_ls"],
                        "rel_res_true": i0["rel_res_true"], "ls_kept": i0["ls_kept"],
                        "seconds": i0["seconds"],
                        "pairwise_iterations": i1["iterations"],
                        "pairwise_used_fallback": i1["used_fallback"],
                        "noise_floor": float(np.linalg.norm(x1 - x0) / np.linalg.norm(x0)),
                        "x_sample": xs0, "x_norm": xn0,
                    }
                    del partial[s]
            json.dump(rec, open(out, "w"))


if __name__ == "__main__":
    main()
