"""Write tests/golden/dense_8192.json from the CPU oracle alone.

The dense FP64 workload: A = G G^T / n + 1e-3 I (n = 8192, G iid N(0,1) on
the 2^-8 grid, so the bytes of A do not depend on the BLAS that forms it),
b ~ N(0,1), no preconditioning, tolerance 1e-8.  For each block width s the
oracle's Algorithm 1, and the Chronopoulos-Gear CG, run in the oracle's three
rounding variants (reference, blocked-pairwise sums, fused multiply-adds).
Stored: iteration counts, exit diagnostics, the noise floor (largest
relative distance between two variants' x), and x at 4096 fixed indices,
plus a hash of the input bytes.

    python tests/golden/make_dense_golden.py [--n 8192] [--s 1,4,8,16,32] [--jobs 6]

Each (s, variant) is one job of a process pool; results are written as
they arrive, and widths already in the output are skipped.
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

import golden_common as G  # noqa: E402
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
    n, kind, s, variant = task
    A, b = system(n)
    t = time.time()
    if kind == "cg":
        x, info, _ = G.run_variant(variant, O.cg_cg, A, b, tol=TOL, jacobi=False)
    else:
        x, info, _ = G.run_variant(variant, O.mbpcg_solve, A, b, s, tol=TOL, jacobi=False,
                                   seed=W.uniform_block_seed(W.CFG_DENSE, s))
    info["seconds_wall"] = time.time() - t
    return task, info, x


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
    idx = sample_index(args.n)
    rec = json.load(open(out)) if os.path.exists(out) else {}
    rec.update({"n": args.n, "shift": 1e-3, "tol": TOL, "input_sha256": input_hash(A, b),
                "sample_index": idx.tolist()})
    rec.setdefault("mbpcg", {})
    keys = [] if "cg" in rec else [("cg", 1)]
    keys += [("mbpcg", s) for s in [int(v) for v in args.s.split(",")]
             if str(s) not in rec["mbpcg"]]
    tasks = [(args.n, kind, s, v) for kind, s in keys for v in G.VARIANTS]
    tasks.sort(key=lambda t: -t[2])   # longest jobs first
    got = {}
    with mp.get_context("fork").Pool(args.jobs) as pool:
        for (n, kind, s, v), info, x in pool.imap_unordered(job, tasks):
            print(kind, s, v, info["iterations"], f"{info['seconds_wall']:.0f} s", flush=True)
            got.setdefault((kind, s), {})[v] = (x, info)
            if len(got[(kind, s)]) < len(G.VARIANTS):
                continue
            runs = got.pop((kind, s))
            if kind == "cg":
                rec["cg"] = G.mbpcg_record(runs, idx)
            else:
                rec["mbpcg"][str(s)] = G.mbpcg_record(runs, idx,
                                                      seed=W.uniform_block_seed(W.CFG_DENSE, s))
            json.dump(rec, open(out, "w"))


if __name__ == "__main__":
    main()
