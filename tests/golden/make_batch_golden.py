"""Write tests/golden/batch_512.json from the CPU oracle alone.

The batched workload: 512 random-graph Laplacians (average degree 8) plus
1e-2 I, n log-uniform in [1e3, 2e5], b ~ N(0,1), block width drawn from
{1, 4, 8}, Jacobi scaling, tolerance 1e-8 (workloads.graph_laplacian_batch).
System i draws its initial block from SplitMix64 seeded with SEED + i, as a
batched solve with common seed SEED does.  For every system the oracle's
Algorithm 1 runs in its three rounding variants (reference, blocked-pairwise
sums, fused multiply-adds); stored per system: n, nnz, s, iteration counts,
exit diagnostics, the noise floor (largest relative distance between two
variants' x), |x|, and x at 16 fixed indices; plus a hash of all input
bytes and the reference runs' total time.

    python tests/golden/make_batch_golden.py [--count 512] [--jobs 6]
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

SEED = 500
_SYS = []


def batch_hash(systems):
    h = hashlib.sha256()
    for y in systems:
        for a in (y.A.rowptr, y.A.colind, y.A.vals, y.b):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(np.int64(y.s).tobytes())
    return h.hexdigest()


def sample_index(i, n, k=16):
    return np.unique(W.rng_for((98, i, n)).integers(0, n, k))


def job(task):
    i, variant = task
    y = _SYS[i]
    x, info, _ = G.run_variant(variant, O.mbpcg_solve, y.A, y.b, y.s, seed=SEED + i)
    return task, info, x


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--jobs", type=int, default=6)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    out = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                   f"batch_{args.count}.json")
    t = time.time()
    _SYS.extend(W.graph_laplacian_batch(count=args.count))
    print(f"generated {len(_SYS)} systems in {time.time() - t:.0f} s", flush=True)
    rec = {"count": args.count, "seed": SEED, "input_sha256": batch_hash(_SYS), "systems": []}
    tasks = [(i, v) for i in range(len(_SYS)) for v in G.VARIANTS]
    res = {}
    with mp.get_context("fork").Pool(args.jobs) as pool:
        for k, ((i, v), info, x) in enumerate(pool.imap_unordered(job, tasks, chunksize=4)):
            res.setdefault(i, {})[v] = (x, info)
            if (k + 1) % 192 == 0:
                print(f"{k + 1}/{len(tasks)} runs", flush=True)
    total = 0.0
    for i, y in enumerate(_SYS):
        idx = sample_index(i, y.A.n)
        total += res[i]["seq"][1]["seconds"]
        r = G.mbpcg_record(res[i], idx, n=y.A.n, nnz=y.A.nnz, s=y.s, seed=SEED + i,
                           sample_index=idx.tolist())
        rec["systems"].append(r)
    rec["oracle_seconds_total"] = total
    json.dump(rec, open(out, "w"))
    print(f"oracle total {total:.0f} s (reference runs, one thread each)", flush=True)


if __name__ == "__main__":
    main()
