"""Autotuner for the launch shape of the BitCol listing kernels.

Searched knobs (kc_options): how many waves share one root's bitmaps in LDS
(lanes per root: 64, 256 or 512), whether candidate sets of at most 64
members are re-encoded into 64-bit rows and from which recursion level (the
width of the bitmaps the deepest levels run on), and how many queue items a
workgroup takes per access (chunking).  None of them changes a result.

The objective is the device time of the listing kernels (HIP events, from the
call's statistics) on the problem itself, or on a cheaper proxy when asked
(the same graph at k-1: about ten times less work, but its best launch shape
can differ).  Decisions are cached in autotune.json next to this module,
keyed by a signature of the graph and k.

Run ``python -m paper_2203_13512_amd.autotune [workload:k ...]`` on a GPU to
tune the synthetic workloads (with the learned schedule when a model for k
exists) and write the cache.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

import paper_2203_13512_amd as kc

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune.json")

SPACE = [
    {},  # library defaults: waves per root by word class, re-encoding up to 128 members from level 4
    {"waves_per_root": 4},
    {"waves_per_root": 8},
    {"compress": 64},
    {"compress_level": 3},
    {"compress_level": 5},
    {"waves_per_root": 8, "compress": 64},
    {"waves_per_root": 8, "class_streams": 2},
]


def signature(row_ptr, col_idx, k: int, order: str) -> str:
    rp = np.asarray(row_ptr.cpu() if hasattr(row_ptr, "cpu") else row_ptr, dtype=np.int32)
    h = hashlib.blake2b(digest_size=12)
    h.update(np.asarray([len(rp) - 1, int(rp[-1]), k], dtype=np.int64).tobytes())
    h.update(order.encode())
    h.update(np.ascontiguousarray(rp[: 1 << 16]).tobytes())
    return h.hexdigest()


def load_cache(path: str = CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(row_ptr, col_idx, k: int, order: str = "color", path: str = CACHE, schedule: str | None = None) -> dict:
    """Tuned kc.count keyword arguments for this graph and k ({} if untuned).
    With `schedule`, the shape tuned under that schedule if there is one, else
    the shape tuned under the other schedule (same kernels, same tuning)."""
    sig = signature(row_ptr, col_idx, k, order)
    cache = load_cache(path)
    keys = ([f"{sig}/{schedule}"] if schedule else []) + [sig]
    keys += [key for key in cache if key.startswith(sig + "/")]
    for key in keys:
        e = cache.get(key)
        if e:
            return dict(e["best"])
    return {}


def tune(row_ptr, col_idx, k: int, order: str = "color", space=SPACE, log=print, proxy: bool = False, **count_kw):
    """Times every candidate (on the k-1 proxy if `proxy`); returns (best, table)."""
    import torch
    kp = k - 1 if (proxy and k >= 4) else k
    table = []
    for cand in space:
        kw = dict(count_kw)
        kw.update(cand)
        torch.cuda.synchronize()
        c, st = kc.count(row_ptr, col_idx, kp, order, stats=True, **kw)
        torch.cuda.synchronize()
        table.append(dict(cand=cand, list_ms=st["list_ms"], total_ms=st["total_ms"], count=c))
        log(f"  k={kp} {cand}: list {st['list_ms']:.1f} ms")
    counts = {t["count"] for t in table}
    assert len(counts) == 1, f"tuning candidates disagree: {counts}"
    best = min(table, key=lambda t: t["list_ms"])["cand"]
    return best, dict(proxy_k=kp, table=table)


def main(argv=None):
    import torch

    import graphgen
    argv = argv if argv is not None else sys.argv[1:]
    from paper_2203_13512_amd import scheduler
    # jobs "workload:k" (learned schedule when a model exists) or "workload:k:degree"
    jobs = [tuple(a.split(":")) for a in argv] or [("5", "8"), ("5", "7"), ("2", "7")]
    cache = load_cache()
    dev = torch.device("cuda:0")
    for job in jobs:
        cfg, k = int(job[0]), int(job[1])
        sched = job[2] if len(job) > 2 else "learned"
        mlp = scheduler.load_model(dev, k) if sched == "learned" else None
        kw = dict(schedule="learned", mlp=mlp) if mlp is not None else {}
        w = graphgen.workload(cfg)
        rp_h, ci_h = w.graphs[0]
        rp = torch.from_numpy(rp_h).to(dev)
        ci = torch.from_numpy(ci_h).to(dev)
        t = time.time()
        print(f"{w.name} k={k}", flush=True)
        best, info = tune(rp, ci, k, "color", **kw)
        sig = signature(rp_h, ci_h, k, "color")
        used = kw.get("schedule", "degree")
        cache[sig if used == "learned" else f"{sig}/{used}"] = dict(workload=w.name, k=k, order="color",
                                                                   schedule=used, best=best, **info)
        print(f"  best {best} ({time.time() - t:.1f}s)", flush=True)
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1)
    out = os.environ.get("KC_AUTOTUNE_OUT")
    if out:
        with open(out, "w") as f:
            json.dump(cache, f, indent=1)


if __name__ == "__main__":
    main()
