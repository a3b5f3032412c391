"""Writes the full-size golden values under tests/golden/ from the CPU oracle.

Only ``oracle/`` computes anything here; ``graphgen/`` supplies the seeded
inputs.  No value comes from the GPU library.

For each job "workload:k:order" (order "color" = BitCol on the degeneracy
DAG, "degree" = SDegree on the degree DAG, Sec. 6-7) the script runs the
oracle's Pre-Core (Alg. 3), Pre-List (Alg. 4) and orientation on the full
workload graph, then the oracle's instrumented listing from every root with
d+ >= k-1, split over worker processes by disjoint root slices (roots are
independent; Theorem 1 makes the count additive over them).  It writes
``fullsize_w<workload>_k<k>_<order>.json`` with the graph's content hash, the
totals, and SHA-256 digests of the per-root arrays indexed by vertex id
(little-endian uint64, zero for vertices that are not roots): the cliques
listed from each root, its joins and its work (BitCol: ceil(s/32) words per
BitJoin; SDegree: |C| + d+ per merge join, the cost of Lemma 2).

For workload 4 ("4:batch") it writes the oracle's count of each of the 256
graphs at its own k to ``fullsize_w4_batch.json``.

Usage: python tests/golden/make_fullsize.py [--procs P] JOB [JOB ...]
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


def graph_sha(rp, ci) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(rp, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(ci, dtype="<i4").tobytes())
    return h.hexdigest()


def array_sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()


_JOB = None


def _slice(i_p):
    i, p = i_p
    drp, dci, k, order, roots = _JOB
    mine = roots[i::p]
    if order == "color":
        per = oracle.bitcol_roots(drp, dci, k, mine)
        return i, per["count"], per["isect"], per["words"], per["nodes"]
    per = oracle.sdegree_roots(drp, dci, k, mine)
    return i, per["count"], per["isect"], per["elems"], per["nodes"]


def run_single(cfg: int, k: int, order: str, procs: int) -> dict:
    global _JOB
    t0 = time.time()
    w = graphgen.workload(cfg)
    rp, ci = w.graphs[0]
    n = len(rp) - 1
    removed = oracle.precore(rp, ci, k)
    removed, pl, _, ncomp = oracle.prelist(rp, ci, k, removed)
    if order == "color":
        drp, dci, _, core = oracle.degeneracy_dag(rp, ci, removed)
    else:
        drp, dci = oracle.degree_dag(rp, ci, removed)
    dplus = np.diff(drp)
    # heaviest first, dealt round-robin: the slices' work stays even
    roots = np.flatnonzero(dplus >= k - 1).astype(np.int32)
    roots = roots[np.argsort(-dplus[roots], kind="stable")]
    print(f"{w.name} k={k} {order}: n={n} prelist={pl} roots={len(roots)} max d+={int(dplus.max())} "
          f"({time.time() - t0:.1f}s)", flush=True)
    _JOB = (drp, dci, k, order, roots)
    parts = 8 * procs
    cnt = np.zeros(n, dtype=np.uint64)
    isect = np.zeros(n, dtype=np.uint64)
    work = np.zeros(n, dtype=np.uint64)
    nodes = 0
    with mp.get_context("fork").Pool(procs) as pool:
        for i, c, j, wk, nd in pool.imap_unordered(_slice, [(i, parts) for i in range(parts)]):
            mine = roots[i::parts]
            cnt[mine], isect[mine], work[mine] = c, j, wk
            nodes += int(nd.sum())
    listing = int(cnt.sum(dtype=np.uint64))
    out = dict(workload=w.name, cfg=cfg, k=k, order=order, n=n, nnz=int(len(ci)), graph_sha256=graph_sha(rp, ci),
               count=listing + pl, prelist_count=pl, listing_count=listing, n_roots=int(len(roots)),
               max_out_degree=int(dplus.max()), isect_total=int(isect.sum(dtype=np.uint64)),
               work_total=int(work.sum(dtype=np.uint64)), nodes_total=nodes,
               per_root_count_sha256=array_sha(cnt), per_root_isect_sha256=array_sha(isect),
               per_root_work_sha256=array_sha(work), oracle_seconds=round(time.time() - t0, 1),
               oracle_processes=procs)
    if order == "color":
        out["max_core"] = int(core.max())
    return out


def run_batch(procs: int) -> dict:
    t0 = time.time()
    w = graphgen.workload(4)
    with mp.get_context("fork").Pool(procs) as pool:
        counts = pool.starmap(oracle.count, [(g[0], g[1], k) for g, k in zip(w.graphs, w.ks)])
    return dict(workload=w.name, cfg=4, ks=[int(k) for k in w.ks], counts=[int(c) for c in counts],
                graph_sha256=[graph_sha(*g) for g in w.graphs], total=int(sum(counts)),
                oracle_seconds=round(time.time() - t0, 1), oracle_processes=procs)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("jobs", nargs="+")
    args = ap.parse_args(argv)
    for job in args.jobs:
        parts = job.split(":")
        if parts[0] == "4":
            out = run_batch(args.procs)
            path = os.path.join(HERE, "fullsize_w4_batch.json")
        else:
            cfg, k, order = int(parts[0]), int(parts[1]), parts[2]
            out = run_single(cfg, k, order, args.procs)
            path = os.path.join(HERE, f"fullsize_w{cfg}_k{k}_{order}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(f"wrote {path}: {json.dumps({key: v for key, v in out.items() if 'sha' not in key})[:400]}",
              flush=True)


if __name__ == "__main__":
    main()
