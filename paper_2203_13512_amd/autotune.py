"""Autotuner for the launch shape of the BitCol listing kernels.

Searched knobs (kc_options, GRID below): how many waves share one root's
bitmaps in LDS (lanes per root: 64, 256, 512 or 1024), how many queue items a
workgroup takes per access (chunking), up to which candidate-set size nodes
are re-encoded into 64-bit rows and from which recursion level (the word
width the deepest levels run on), and whether the word classes' kernels run
in sequence or concurrently.  None of them changes a result.  The search is a
coordinate descent (one knob at a time, the others at the best so far).

The objective is the device time of the listing kernels (HIP events, from the
call's statistics) on the problem itself, or on a cheaper proxy when asked
(the same graph at k-1: about ten times less work, but its best launch shape
can differ); for a batch of graphs, the replay time of its captured plan.
Decisions are cached in autotune.json next to this module, keyed by a
signature of the graph and k (and the schedule, for the degree schedule).

Run ``python -m paper_2203_13512_amd.autotune [workload:k[:degree][:proxy] | 4 ...]``
on a GPU to tune the synthetic workloads (with the learned schedule when a
model for k exists) and write the cache.
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

# The search grid (kc_options knobs; 0 = the library's default for the knob):
# lanes per root (waves sharing one root's bitmaps: 1, 4, 8 -> 64, 256, 512
# lanes), work items per queue access, the largest candidate set re-encoded
# into 64-bit rows (which sets the word width the deepest levels run on: 32-bit
# words of the full bitmaps, or one or two 64-bit words), the lowest level
# re-encoded, and whether the word classes' kernels run in sequence or
# concurrently.
GRID = {
    "waves_per_root": [0, 1, 4, 8, 16],
    "chunk": [0, 1, 4, 16, 64],
    "compress": [0, 64, -1],
    "compress_level": [0, 3, 5],
    "class_streams": [1, 2],
}
def coordinate_descent(evaluate, grid=GRID, start=None, sweeps: int = 1, log=print):
    """Minimises evaluate(candidate) over the grid one knob at a time: each
    knob takes every value with the others held at the best so far; repeated
    for `sweeps` passes.  Returns (best candidate, {candidate key: time})."""
    best = dict(start or {})
    seen = {}

    def key(c):
        return tuple(sorted((k, v) for k, v in c.items() if v != 0))

    def run(c):
        kk = key(c)
        if kk not in seen:
            seen[kk] = evaluate({k: v for k, v in c.items() if v != 0})
            log(f"  {dict(kk)}: {seen[kk]:.1f} ms")
        return seen[kk]

    t_best = run(best)
    for _ in range(sweeps):
        for knob, values in grid.items():
            for v in values:
                cand = dict(best)
                cand[knob] = v
                t = run(cand)
                if t < t_best:
                    best, t_best = cand, t
    return {k: v for k, v in best.items() if v != 0}, {str(dict(k)): t for k, t in seen.items()}


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


def tune(row_ptr, col_idx, k: int, order: str = "color", log=print, proxy: bool = False, sweeps: int = 1,
         **count_kw):
    """Coordinate descent over GRID on the listing time (HIP events of the
    call's listing kernels), on the k-1 proxy if `proxy`; every candidate must
    give the same count.  Returns (best, info)."""
    import torch
    kp = k - 1 if (proxy and k >= 4) else k
    counts = set()

    def evaluate(cand):
        kw = dict(count_kw)
        kw.update(cand)
        torch.cuda.synchronize()
        c, st = kc.count(row_ptr, col_idx, kp, order, stats=True, **kw)
        torch.cuda.synchronize()
        counts.add(c)
        return st["list_ms"]

    best, table = coordinate_descent(evaluate, sweeps=sweeps, log=log)
    assert len(counts) == 1, f"tuning candidates disagree: {counts}"
    return best, dict(proxy_k=kp, list_ms=table, count=counts.pop())


def tune_batched(graphs, ks, log=print, replays: int = 3, **plan_kw):
    """The same search for a batch of graphs on the captured plan's replay
    time (median of `replays` executions); every replay must give the same
    per-graph counts.  Returns (best, info)."""
    import statistics
    import time
    results = set()

    def evaluate(cand):
        kw = dict(plan_kw)
        kw.update(cand)
        kw.pop("class_streams", None)  # a plan's listing phase is one chain of kernels
        plan = kc.plan_batched(graphs, ks, "color", **kw)
        try:
            ts = []
            for _ in range(replays):
                t0 = time.perf_counter()
                results.add(tuple(plan.execute()))
                ts.append((time.perf_counter() - t0) * 1e3)
        finally:
            plan.close()
        return statistics.median(ts)

    grid = {key: v for key, v in GRID.items() if key != "class_streams"}
    best, table = coordinate_descent(evaluate, grid=grid, log=log)
    assert len(results) == 1, "tuning candidates disagree"
    return best, dict(replay_ms=table)


def batch_signature(graphs, ks) -> str:
    h = hashlib.blake2b(digest_size=12)
    for (rp, ci), k in zip(graphs, ks):
        h.update(signature(rp, ci, int(k), "color").encode())
    return "batch-" + h.hexdigest()


def main(argv=None):
    import torch

    import graphgen
    argv = argv if argv is not None else sys.argv[1:]
    from paper_2203_13512_amd import scheduler
    # jobs "workload:k" (learned schedule when a model exists), "workload:k:degree",
    # optionally ":proxy" (tune at k-1), or "4" (the batch of graphs, plan replays)
    jobs = [tuple(a.split(":")) for a in argv] or [("5", "8"), ("5", "7"), ("2", "7")]
    cache = load_cache()
    dev = torch.device("cuda:0")
    for job in jobs:
        if job[0] == "4":
            w = graphgen.workload(4)
            t = time.time()
            print(f"{w.name}: {len(w.graphs)} graphs", flush=True)
            best, info = tune_batched(w.graphs, w.ks)
            cache[batch_signature(w.graphs, w.ks)] = dict(workload=w.name, k=0, order="color", schedule="degree",
                                                          best=best, **info)
            print(f"  best {best} ({time.time() - t:.1f}s)", flush=True)
            with open(CACHE, "w") as f:
                json.dump(cache, f, indent=1)
            continue
        cfg, k = int(job[0]), int(job[1])
        sched = job[2] if len(job) > 2 and job[2] != "proxy" else "learned"
        proxy = "proxy" in job
        mlp = scheduler.load_model(dev, k) if sched == "learned" else None
        kw = dict(schedule="learned", mlp=mlp) if mlp is not None else {}
        w = graphgen.workload(cfg)
        rp_h, ci_h = w.graphs[0]
        rp = torch.from_numpy(rp_h).to(dev)
        ci = torch.from_numpy(ci_h).to(dev)
        t = time.time()
        print(f"{w.name} k={k}", flush=True)
        best, info = tune(rp, ci, k, "color", proxy=proxy, **kw)
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
