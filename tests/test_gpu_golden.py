"""Full-size parity against golden values written by the CPU oracle
(tests/golden/make_fullsize.py calls only oracle/ on the seeded workloads).

For each stored workload, k and order the GPU run must give the oracle's
total and Pre-List count and, root by root over the whole graph, the same
cliques listed from each root, the same joins and the same work (compared as
SHA-256 digests of the per-vertex arrays).  BitCol runs in the benchmark's
launch configuration (learned schedule, tuned launch shape) and under the
degree schedule; these workloads put roots into the 8-, 12- and 16-word
bitmap classes, which carry most of the benchmark's listing time.  Workloads
beyond the oracle's full enumeration are checked on sampled roots of every
wide word class (tests/golden/make_sampled.py).  The batched workload (256
graphs with their own k) is checked graph by graph, eagerly and through
every replay of a prepared plan.
"""
import glob
import json
import os
import sys

import numpy as np
import pytest

import oracle
from tests import _graphs as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2203_13512_amd as kc  # noqa: E402
from paper_2203_13512_amd import autotune, scheduler  # noqa: E402

SINGLE = sorted(glob.glob(os.path.join(G.GOLDEN, "fullsize_w[0-9]_k*_*.json")))
BATCH = os.path.join(G.GOLDEN, "fullsize_w4_batch.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _load(path):
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("path", SINGLE, ids=[os.path.basename(p)[:-5] for p in SINGLE])
def test_fullsize_per_root_parity(path):
    gd = _load(path)
    w = G.workload_cached(gd["cfg"])
    rp_h, ci_h = w.graphs[0]
    assert G.graph_sha(rp_h, ci_h) == gd["graph_sha256"], "the generator no longer makes the stored graph"
    k, order = gd["k"], gd["order"]
    rp = torch.from_numpy(rp_h).cuda()
    ci = torch.from_numpy(ci_h).cuda()
    # vertices that Pre-List removes (clique components): the smallest one of
    # each carries the component's C(n_c, k) in the per-root attribution
    removed = oracle.precore(rp_h, ci_h, k)
    after, pl, _, _ = oracle.prelist(rp_h, ci_h, k, removed)
    assert pl == gd["prelist_count"]
    pl_mask = (after != 0) & (removed == 0)
    runs = [dict()]
    if order == "color":
        tuned = autotune.lookup(rp_h, ci_h, k, order, schedule="learned")
        runs = [dict(schedule="learned", mlp=scheduler.load_model(rp.device, k), **tuned),
                dict(schedule="degree", **tuned)]
    for kw in runs:
        say(os.path.basename(path), {key: v for key, v in kw.items() if key != "mlp"})
        c, st = kc.count(rp, ci, k, order, root_logs=True, **kw)
        lg = {key: v.cpu().numpy() for key, v in st["root_logs"].items()}
        assert c == gd["count"]
        assert st["prelist_count"] == gd["prelist_count"]
        assert st["n_roots"] == gd["n_roots"] and st["max_out_degree"] == gd["max_out_degree"]
        cnt = lg["count"].astype(np.uint64)
        assert int(cnt[pl_mask].sum()) == gd["prelist_count"]
        cnt[pl_mask] = 0
        assert G.array_sha(cnt) == gd["per_root_count_sha256"]
        assert G.array_sha(lg["isect"].astype(np.uint64)) == gd["per_root_isect_sha256"]
        assert G.array_sha(lg["work"].astype(np.uint64)) == gd["per_root_work_sha256"]
        assert st["isect"] == gd["isect_total"] and st["work"] == gd["work_total"]
        assert st["nodes"] == gd["nodes_total"]
        if order == "color":
            assert st["max_core"] == gd["max_core"]


SAMPLED = sorted(glob.glob(os.path.join(G.GOLDEN, "sampled_w[0-9]_k*_color.json")))


@pytest.mark.parametrize("path", SAMPLED, ids=[os.path.basename(p)[:-5] for p in SAMPLED])
def test_sampled_root_parity(path):
    """Workloads whose full enumeration is beyond the oracle: the cliques,
    BitJoins and words of the cheapest roots of the 8-, 12-, 16- and
    24-word classes (tests/golden/make_sampled.py), from the GPU run
    restricted to those roots (kc_options.root_mask) and, where the whole
    workload takes seconds (k <= 6), from the whole run."""
    gd = _load(path)
    w = G.workload_cached(gd["cfg"])
    rp_h, ci_h = w.graphs[0]
    assert G.graph_sha(rp_h, ci_h) == gd["graph_sha256"], "the generator no longer makes the stored graph"
    k = gd["k"]
    rp = torch.from_numpy(rp_h).cuda()
    ci = torch.from_numpy(ci_h).cuda()
    roots = np.asarray(gd["roots"], dtype=np.int64)
    mask = torch.zeros(len(rp_h) - 1, dtype=torch.bool, device=rp.device)
    mask[torch.from_numpy(roots).to(rp.device)] = True
    tuned = autotune.lookup(rp_h, ci_h, k, "color", schedule="learned")
    for kw in (dict(schedule="learned", mlp=scheduler.load_model(rp.device, k), **tuned), dict(schedule="degree")):
        for whole in ((False, True) if k <= 6 else (False,)):
            say(os.path.basename(path), "whole run" if whole else "sampled roots only",
                {key: v for key, v in kw.items() if key != "mlp"})
            c, st = kc.count(rp, ci, k, "color", root_logs=True, root_mask=None if whole else mask, **kw)
            lg = {key: v.cpu().numpy() for key, v in st["root_logs"].items()}
            assert np.array_equal(lg["features"][roots, 0].astype(np.int64), gd["out_degree"])
            assert np.array_equal(lg["features"][roots, 1].astype(np.int64), gd["core"])
            assert np.array_equal(lg["count"][roots], np.asarray(gd["count"], dtype=np.int64))
            assert np.array_equal(lg["isect"][roots], np.asarray(gd["isect"], dtype=np.int64))
            assert np.array_equal(lg["work"][roots], np.asarray(gd["words"], dtype=np.int64))
            assert int(lg["count"].sum()) == c
            if whole:
                assert st["prelist_count"] == gd["prelist_count"]
            else:
                # the sampled roots are DAG roots, none the smallest vertex of
                # a clique component
                assert st["n_roots"] == len(roots) and st["prelist_count"] == 0
                assert c == sum(gd["count"])


@pytest.mark.skipif(not os.path.exists(BATCH), reason="no stored batch counts")
def test_fullsize_batch_eager_and_replayed():
    gd = _load(BATCH)
    w = G.workload_cached(4)
    assert [G.graph_sha(*g) for g in w.graphs] == gd["graph_sha256"]
    assert list(w.ks) == gd["ks"]
    want = gd["counts"]
    for order in ("color", "degree"):
        say("batch", len(w.graphs), order)
        assert kc.count_batched(w.graphs, w.ks, order) == want, order
    mlp = scheduler.load_model(torch.device("cuda"), 8)
    for kw in [dict(), dict(schedule="learned", mlp=mlp, waves_per_root=8)]:
        say("batch plan", {key: v for key, v in kw.items() if key != "mlp"})
        plan = kc.plan_batched(w.graphs, w.ks, "color", **kw)
        try:
            for i in range(3):
                assert plan.execute() == want, i
                torch.cuda.synchronize()
        finally:
            plan.close()
