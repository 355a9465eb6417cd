"""Write tests/golden/dense_mixed_16384.json from the CPU oracle alone.

The mixed-precision dense workload: A = G G^T / n + 1e-3 I (n = 16384, G
iid N(0,1) on the 2^-8 grid, so A's bytes do not depend on the BLAS),
b ~ N(0,1), no preconditioning.  Stored:

* an FP64 reference solution: the oracle's Algorithm 1 at s = 8 to the
  relative residual 1e-12, cross-checked against numpy.linalg.solve (LAPACK
  LU) -- x at 4096 fixed indices, its norm, and the relative difference of
  the two solutions;
* for s in {8, 16, 32}: the oracle's iterative refinement to 1e-10 with FP32
  inner products emulated (A and the blocks rounded to FP32, products
  accumulated in FP32), i.e. the arithmetic of the GPU's FP32 path, once
  with sequential FP32 sums over the 16384 columns ("ir_fp32") and once
  with blocked-pairwise FP32 sums ("ir_fp32_pairwise") -- outer and inner
  iteration counts, the FP64 residual, the error against the reference, and
  sampled x.

    python tests/golden/make_dense_mixed_golden.py [--n 16384] [--s 8,16,32] [--jobs 4]

A is formed once, kept in /dev/shm for the worker processes while they run,
and removed at the end.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2608_07327_amd import workloads as W  # noqa: E402

REF_S = 8
REF_TOL = 1e-12
IR_TOL = 1e-10
INNER_TOL = 5e-6


def sample_index(n, k=4096):
    return np.unique(W.rng_for((99, n)).integers(0, n, k))


def job(task):
    path, n, kind, s = task
    A = np.load(path, mmap_mode="r")
    b = W.rhs(n, W.CFG_DENSE_MIXED)
    seed = W.uniform_block_seed(W.CFG_DENSE_MIXED, s)
    t = time.time()
    O.set_variant("pairwise" if kind == "ir_pairwise" else "seq")
    if kind == "ref":
        # A is symmetric: its transpose view is the column-major matrix, no copy
        x, info, _ = O.mbpcg_solve(np.asarray(A).T, b, s, tol=REF_TOL, jacobi=False, seed=seed)
    else:
        x, info = O.ir_solve(np.asarray(A).T, b, s, O.LO_FP32, ir_tol=IR_TOL,
                             inner_tol=INNER_TOL, seed=seed)
    info["seconds_wall"] = time.time() - t
    return task, info, x


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--s", default="8,16,32")
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--out", default=None)
    ap.add_argument("--kinds", default="ref,ir,ir_pairwise",
                    help="which runs to add when missing from the output")
    args = ap.parse_args()
    kinds = set(args.kinds.split(","))
    n = args.n
    out = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                   f"dense_mixed_{n}.json")
    t = time.time()
    A = W.dense_spd(n, W.CFG_DENSE_MIXED)
    b = W.rhs(n, W.CFG_DENSE_MIXED)
    h = hashlib.sha256()
    h.update(A.tobytes())
    h.update(b.tobytes())
    idx = sample_index(n)
    rec = json.load(open(out)) if os.path.exists(out) else {}
    rec.update({"n": n, "shift": 1e-3, "input_sha256": h.hexdigest(),
                "sample_index": idx.tolist(), "ref_s": REF_S, "ref_tol": REF_TOL,
                "ir_tol": IR_TOL, "inner_tol": INNER_TOL})
    rec.setdefault("ir_fp32", {})
    rec.setdefault("ir_fp32_pairwise", {})
    print(f"inputs {time.time() - t:.0f} s", flush=True)
    x_np = None
    if "ref" not in rec and "ref" in kinds:
        t = time.time()
        x_np = np.linalg.solve(A, b)
        print(f"numpy solve {time.time() - t:.0f} s", flush=True)
    path = f"/dev/shm/mbpcg_golden_dense_{n}_{os.getpid()}.npy"
    np.save(path, A)
    del A
    tasks = [] if ("ref" in rec or "ref" not in kinds) else [(path, n, "ref", REF_S)]
    widths = [int(v) for v in args.s.split(",")]
    if "ir" in kinds:
        tasks += [(path, n, "ir", s) for s in widths if str(s) not in rec["ir_fp32"]]
    if "ir_pairwise" in kinds:
        tasks += [(path, n, "ir_pairwise", s) for s in widths
                  if str(s) not in rec["ir_fp32_pairwise"]]
    tasks.sort(key=lambda q: -q[3])
    x_ref = None
    irs = {}
    import multiprocessing as mp
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        with mp.get_context("spawn").Pool(args.jobs) as pool:
            for (_, _, kind, s), info, x in pool.imap_unordered(job, tasks):
                print(kind, s, info.get("iterations"), f"{info['seconds_wall']:.0f} s", flush=True)
                if kind == "ref":
                    x_ref = x
                    rec["ref"] = {
                        "seed": W.uniform_block_seed(W.CFG_DENSE_MIXED, s),
                        "iterations": info["iterations"], "status": info["status"],
                        "used_fallback": info["used_fallback"],
                        "rel_res_true": info["rel_res_true"], "x_sample": x[idx].tolist(),
                        "x_norm": float(np.linalg.norm(x)),
                        "vs_numpy_solve": float(np.linalg.norm(x - x_np) / np.linalg.norm(x_np)),
                        "numpy_x_sample": x_np[idx].tolist(),
                    }
                    for (key, s2), (i2, x2) in list(irs.items()):
                        rec[key][str(s2)]["err_vs_ref"] = float(
                            np.linalg.norm(x2 - x_ref) / np.linalg.norm(x_ref))
                else:
                    key = "ir_fp32" if kind == "ir" else "ir_fp32_pairwise"
                    irs[(key, s)] = (info, x)
                    rec[key][str(s)] = {
                        "seed": W.uniform_block_seed(W.CFG_DENSE_MIXED, s),
                        "outer_iterations": info["outer_iterations"],
                        "iterations": info["iterations"],
                        "inner_iterations": info["inner_iterations"],
                        "status": info["status"], "rel_res_true": info["rel_res_true"],
                        "x_sample": x[idx].tolist(),
                        "err_vs_ref": (float(np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref))
                                       if x_ref is not None else None),
                    }
                    if x_ref is None and "ref" in rec:
                        # the reference of an earlier invocation: its sampled entries
                        xr = np.asarray(rec["ref"]["x_sample"])
                        rec[key][str(s)]["err_vs_ref_sampled"] = float(
                            np.linalg.norm(x[idx] - xr) / np.linalg.norm(xr))
                json.dump(rec, open(out, "w"))
    finally:
        os.unlink(path)


if __name__ == "__main__":
    main()
