"""Write tests/golden/diffusion3d_128.json from the CPU oracle alone.

For the 128^3 diffusion system (seeded inputs from the workload module) and
each block width s, the oracle's Algorithm 1 runs in its three rounding
variants (reference, blocked-pairwise sums, fused multiply-adds), and the
Chronopoulos-Gear CG likewise.  Stored: iteration counts, exit diagnostics,
the noise floor (largest relative distance between two variants' x), and x
at 4096 fixed indices, plus a hash of the inputs so a reader can tell
whether its inputs are the same bytes.

    python tests/golden/make_diffusion3d_golden.py [--grid 128] [--s 1,2,4,8,16] [--jobs 6]

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

_SYS = {}


def input_hash(A, b):
    h = hashlib.sha256()
    for a in (A.rowptr, A.colind, A.vals, b):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def sample_index(n, k=4096):
    return np.unique(W.rng_for((99, n)).integers(0, n, k))


def job(task):
    kind, s, variant = task
    A, b = _SYS["A"], _SYS["b"]
    t = time.time()
    if kind == "cg":
        x, info, _ = G.run_variant(variant, O.cg_cg, A, b)
    else:
        x, info, _ = G.run_variant(variant, O.mbpcg_solve, A, b, s,
                                   seed=W.uniform_block_seed(W.CFG_DIFFUSION3D, s))
    info["seconds_wall"] = time.time() - t
    return task, info, x


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--s", default="1,2,4,8,16")
    ap.add_argument("--jobs", type=int, default=6)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    out = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                   f"diffusion3d_{args.grid}.json")
    A = W.diffusion3d(args.grid)
    b = W.rhs(A.n, W.CFG_DIFFUSION3D)
    _SYS.update(A=O.Matrix(A), b=b)
    idx = sample_index(A.n)
    rec = json.load(open(out)) if os.path.exists(out) else {}
    rec.update({"grid": args.grid, "n": A.n, "nnz": A.nnz, "input_sha256": input_hash(A, b),
                "sample_index": idx.tolist()})
    rec.setdefault("mbpcg", {})
    keys = [] if "cg" in rec else [("cg", 1)]
    keys += [("mbpcg", s) for s in [int(v) for v in args.s.split(",")]
             if str(s) not in rec["mbpcg"]]
    tasks = [(kind, s, v) for kind, s in keys for v in G.VARIANTS]
    tasks.sort(key=lambda t: -t[1])   # longest jobs first
    got = {}
    with mp.get_context("fork").Pool(args.jobs) as pool:
        for (kind, s, v), info, x in pool.imap_unordered(job, tasks):
            print(kind, s, v, info["iterations"], f"{info['seconds_wall']:.0f} s", flush=True)
            got.setdefault((kind, s), {})[v] = (x, info)
            if len(got[(kind, s)]) < len(G.VARIANTS):
                continue
            runs = got.pop((kind, s))
            if kind == "cg":
                rec["cg"] = G.mbpcg_record(runs, idx)
            else:
                rec["mbpcg"][str(s)] = G.mbpcg_record(
                    runs, idx, seed=W.uniform_block_seed(W.CFG_DIFFUSION3D, s))
            json.dump(rec, open(out, "w"))


if __name__ == "__main__":
    main()
