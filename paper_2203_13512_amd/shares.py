"""Counting in root shares.

Theorem 1 gives every k-clique exactly one root, its first vertex in the
orientation, so a count is the sum of the counts listed from any partition of
the roots (plus the Pre-List cliques of each clique component, which belong to
the share of its smallest vertex).  ``kc_options.root_mask`` restricts a call
to one share; this module partitions the vertices into S shares by a
multiplicative hash of their ids (heavy and light roots spread evenly) and
runs one call per share.  That splits a count whose single call would run too
long into calls of bounded length, and a share is the unit a run over several
processes or GPUs would hand out.

    python -m paper_2203_13512_amd.shares --workload 3 --k 8 --shares 16 [--range 0:8]

runs shares [a, b) of the seeded workload (learned schedule, tuned launch
shape), prints one JSON line per share as it finishes and a summary line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def share_index(n: int, shares: int, device):
    """int64 tensor of n entries: the share of each vertex, the top bits of
    the 32-bit product of its id with 2654435761 (Knuth's multiplicative
    hash) scaled to [0, shares)."""
    import torch
    u = torch.arange(n, dtype=torch.int64, device=device)
    return ((u * 2654435761) & 0xFFFFFFFF) * shares >> 32


def count_in_shares(row_ptr, col_idx, k: int, order: str = "color", shares: int = 8, which=None, on_share=None,
                    **kw):
    """Counts the graph (CUDA int32 CSR tensors) one share at a time.
    ``which``: the share indices to run (default all); ``on_share(record)``
    is called after each.  Returns the per-share records (share, count, wall
    seconds, the call's statistics)."""
    import torch

    import paper_2203_13512_amd as kc
    if shares < 1:
        raise ValueError("shares must be >= 1")
    which = list(range(shares) if which is None else which)
    if any(not 0 <= s < shares for s in which):
        raise ValueError(f"share indices must lie in [0, {shares})")
    if "stats" in kw or "root_mask" in kw:
        raise TypeError("count_in_shares sets stats and root_mask itself")
    n = row_ptr.numel() - 1
    idx = share_index(n, shares, row_ptr.device)
    out = []
    for s in which:
        mask = idx == s
        torch.cuda.synchronize(row_ptr.device)
        t = time.perf_counter()
        c, st = kc.count(row_ptr, col_idx, k, order, stats=True, root_mask=mask, **kw)
        torch.cuda.synchronize(row_ptr.device)
        rec = dict(share=int(s), of=shares, count=int(c), wall_s=time.perf_counter() - t, stats=st)
        out.append(rec)
        if on_share is not None:
            on_share(rec)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", type=int, required=True)
    ap.add_argument("--k", type=int, required=True)
    ap.add_argument("--order", default="color")
    ap.add_argument("--schedule", default="learned")
    ap.add_argument("--shares", type=int, default=16)
    ap.add_argument("--range", default="", help="a:b, the shares to run (default all)")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch

    import graphgen
    from paper_2203_13512_amd import autotune, scheduler

    w = graphgen.workload(args.workload)
    rp_h, ci_h = w.graphs[0]
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(rp_h).to(dev)
    ci = torch.from_numpy(ci_h).to(dev)
    kw = dict(schedule=args.schedule, class_streams=1)
    if args.schedule == "learned":
        kw["mlp"] = scheduler.load_model(dev, args.k)
    if args.order == "color":
        kw.update({a: b for a, b in autotune.lookup(rp_h, ci_h, args.k, args.order,
                                                     schedule=args.schedule).items() if a not in kw})
    a, b = (int(x) for x in args.range.split(":")) if args.range else (0, args.shares)
    launch = {key: v for key, v in kw.items() if key != "mlp"}
    print(json.dumps({"workload": w.name, "n": int(len(rp_h) - 1), "nnz": int(len(ci_h)), "k": args.k,
                      "order": args.order, "launch": launch, "shares": args.shares, "range": [a, b]}), flush=True)

    def show(r):
        st = r["stats"]
        print(json.dumps({"share": r["share"], "of": r["of"], "count": r["count"], "wall_s": round(r["wall_s"], 3),
                          "list_ms": round(st["list_ms"], 1), "prep_ms": round(st["prep_ms"], 1),
                          "n_roots": st["n_roots"], "n_tasks": st["n_tasks"],
                          "class_ms": [round(x, 1) for x in st["class_ms"]]}), flush=True)

    recs = count_in_shares(rp, ci, args.k, args.order, args.shares, range(a, b), show, **kw)
    print(json.dumps({"summary": True, "shares_run": [a, b], "of": args.shares,
                      "count": sum(r["count"] for r in recs), "wall_s": round(sum(r["wall_s"] for r in recs), 3),
                      "list_ms": round(sum(r["stats"]["list_ms"] for r in recs), 1),
                      "max_share_wall_s": round(max(r["wall_s"] for r in recs), 3)}), flush=True)


if __name__ == "__main__":
    main()
