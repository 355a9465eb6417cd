"""Write tests/golden/diffusion3d_128.json from the CPU oracle alone.

For the 128^3 diffusion system (seeded inputs from the workload module) and
each block width s, the oracle's Algorithm 1 is run twice -- sequential and
blocked-pairwise reductions -- and the Chronopoulos-Gear CG once.  Stored:
iteration counts, exit diagnostics, the rounding-order noise floor
|x_pairwise - x| / |x|, and x at 4096 fixed indices, plus a hash of the
inputs so a reader can tell whether its inputs are the same bytes.

    python tests/golden/make_diffusion3d_golden.py [--grid 128] [--s 1,2,4,8,16]
    python tests/golden/make_diffusion3d_golden.py --merge OTHER.json

--merge takes the block widths of another output of this script (written
with --out, e.g. by a second process running other widths) whose input hash
matches.
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


def input_hash(A, b):
    h = hashlib.sha256()
    for a in (A.rowptr, A.colind, A.vals, b):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def sample_index(n, k=4096):
    return np.unique(W.rng_for((99, n)).integers(0, n, k))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--s", default="1,2,4,8,16")
    ap.add_argument("--out", default=None)
    ap.add_argument("--merge", default=None)
    args = ap.parse_args()
    out = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                   f"diffusion3d_{args.grid}.json")
    A = W.diffusion3d(args.grid)
    b = W.rhs(A.n, W.CFG_DIFFUSION3D)
    M = O.Matrix(A)
    idx = sample_index(A.n)
    rec = json.load(open(out)) if os.path.exists(out) else {}
    rec.update({"grid": args.grid, "n": A.n, "nnz": A.nnz, "input_sha256": input_hash(A, b),
                "sample_index": idx.tolist()})
    rec.setdefault("mbpcg", {})
    if args.merge:
        other = json.load(open(args.merge))
        if other.get("input_sha256") != rec["input_sha256"] or other.get("sample_index") != rec["sample_index"]:
            sys.exit("merge: inputs differ")
        for k, v in other.get("mbpcg", {}).items():
            rec["mbpcg"].setdefault(k, v)
        json.dump(rec, open(out, "w"))
        print("merged widths", sorted(rec["mbpcg"], key=int), flush=True)
        return
    if "cg" not in rec:
        t = time.time()
        x, info, _ = O.cg_cg(M, b)
        rec["cg"] = {"iterations": info["iterations"], "rel_res_true": info["rel_res_true"],
                     "seconds": time.time() - t, "x_sample": x[idx].tolist(),
                     "x_norm": float(np.linalg.norm(x))}
        json.dump(rec, open(out, "w"))
        print("cg", rec["cg"]["iterations"], flush=True)
    for s in [int(v) for v in args.s.split(",")]:
        if str(s) in rec["mbpcg"]:
            continue
        seed = W.uniform_block_seed(W.CFG_DIFFUSION3D, s)
        t = time.time()
        O.set_summation(0)
        x0, i0, _ = O.mbpcg_solve(M, b, s, seed=seed)
        t0 = time.time() - t
        O.set_summation(1)
        x1, i1, _ = O.mbpcg_solve(M, b, s, seed=seed)
        O.set_summation(0)
        rec["mbpcg"][str(s)] = {
            "seed": seed, "iterations": i0["iterations"], "status": i0["status"],
            "best_column": i0["best_column"], "final_width": i0["final_width"],
            "deflations": i0["deflations"], "used_fallback": i0["used_fallback"],
            "rel_res_best": i0["rel_res_best"], "rel_res_ls": i0["rel_res_ls"],
            "rel_res_true": i0["rel_res_true"], "seconds": t0,
            "pairwise_iterations": i1["iterations"],
            "noise_floor": float(np.linalg.norm(x1 - x0) / np.linalg.norm(x0)),
            "x_sample": x0[idx].tolist(), "x_norm": float(np.linalg.norm(x0)),
        }
        json.dump(rec, open(out, "w"))
        print("s", s, i0["iterations"], i1["iterations"], rec["mbpcg"][str(s)]["noise_floor"],
              flush=True)


if __name__ == "__main__":
    main()
