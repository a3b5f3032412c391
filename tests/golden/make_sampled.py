"""Writes golden per-root values for sampled roots of a full-size workload,
from the CPU oracle (for configurations whose full enumeration is out of the
oracle's reach).

Only ``oracle/`` computes anything here; ``graphgen/`` supplies the seeded
input.  No value comes from the GPU library.

For a job "workload:k" the script runs the oracle's Pre-Core (Alg. 3),
Pre-List (Alg. 4) and degeneracy orientation on the full workload graph and
picks, in each bitmap word class of 8, 12, 16 and 24 words (out-degree in
(128, 256], (256, 384], (384, 512], (512, 768]), the `per` roots of smallest
core number (ties by id): the cheapest roots of the class for the oracle.
For each it runs the oracle's BitCol (Alg. 6) from that root alone and
records the cliques listed from it, its BitJoins and its words.  Output:
``sampled_w<workload>_k<k>_color.json``.

Usage: python tests/golden/make_sampled.py [--per N] [--procs P] [--classes 8,12,16,24] [--tag T] JOB [JOB ...]

The file is rewritten as roots finish (in the order of the picks), so a run
cut short keeps the roots it completed.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

CLASSES = {8: (128, 256), 12: (256, 384), 16: (384, 512), 24: (512, 768)}
_JOB = None


def _one(r):
    drp, dci, k = _JOB
    per = oracle.bitcol_roots(drp, dci, k, np.array([r], dtype=np.int32))
    return int(r), int(per["count"][0]), int(per["isect"][0]), int(per["words"][0])


def main():
    global _JOB
    ap = argparse.ArgumentParser()
    ap.add_argument("--per", type=int, default=4)
    ap.add_argument("--procs", type=int, default=4)
    ap.add_argument("--classes", default="8,12,16,24", help="word classes to sample")
    ap.add_argument("--tag", default="", help="written to sampled_w<workload>_k<k>_<tag>_color.json")
    ap.add_argument("jobs", nargs="+")
    args = ap.parse_args()
    for job in args.jobs:
        cfg, k = (int(x) for x in job.split(":"))
        w = graphgen.workload(cfg)
        rp, ci = w.graphs[0]
        t0 = time.time()
        removed = oracle.precore(rp, ci, k)
        removed, pl, _, _ = oracle.prelist(rp, ci, k, removed)
        drp, dci, _, core = oracle.degeneracy_dag(rp, ci, removed)
        dp = np.diff(drp)
        picks = []
        for c in (int(x) for x in args.classes.split(",")):
            lo, hi = CLASSES[c]
            cls = np.flatnonzero((dp > lo) & (dp <= hi))
            picks += [int(r) for r in cls[np.lexsort((cls, core[cls]))][: args.per]]
        _JOB = (drp, dci, k)
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(rp, dtype="<i4").tobytes())
        h.update(np.ascontiguousarray(ci, dtype="<i4").tobytes())
        path = os.path.join(HERE, f"sampled_w{cfg}_k{k}{'_' + args.tag if args.tag else ''}_color.json")
        done = {}
        with mp.get_context("fork").Pool(args.procs) as pool:
            for r in pool.imap_unordered(_one, picks):
                done[r[0]] = r
                res = [done[p] for p in picks if p in done]
                out = {
                    "workload": w.name, "cfg": cfg, "k": k, "order": "color", "n": int(len(rp) - 1),
                    "nnz": int(len(ci)), "graph_sha256": h.hexdigest(), "prelist_count": pl,
                    "roots": [r[0] for r in res], "out_degree": [int(dp[r[0]]) for r in res],
                    "core": [int(core[r[0]]) for r in res], "count": [r[1] for r in res],
                    "isect": [r[2] for r in res], "words": [r[3] for r in res],
                    "oracle_seconds": round(time.time() - t0, 1), "oracle_processes": args.procs,
                }
                with open(path, "w") as f:
                    json.dump(out, f, indent=1)
                print(path, len(res), "of", len(picks), "roots", out["oracle_seconds"], "s", flush=True)


if __name__ == "__main__":
    main()
