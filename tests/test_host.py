"""Host-side logic that needs no GPU: the autotuner's cache keys, the saved
scheduler model, the benchmark's argument contract and the generators'
determinism and recipes."""
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_2203_13512_amd as kc
from paper_2203_13512_amd import autotune, scheduler

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_autotune_signature_is_stable_and_keyed(tmp_path):
    g = graphgen.chung_lu(2000, 8.0, 2.1, 200.0, seed=1)
    s = autotune.signature(*g, 5, "color")
    assert s == autotune.signature(*g, 5, "color")
    assert s != autotune.signature(*g, 6, "color")
    assert s != autotune.signature(*g, 5, "degree")
    h = graphgen.chung_lu(2000, 8.0, 2.1, 200.0, seed=2)
    assert s != autotune.signature(*h, 5, "color")
    assert autotune.lookup(*g, 5, "color", path=str(tmp_path / "none.json")) == {}
    cache = tmp_path / "c.json"
    cache.write_text(json.dumps({s: {"best": {"waves_per_root": 8}}}))
    assert autotune.lookup(*g, 5, "color", path=str(cache)) == {"waves_per_root": 8}


def test_autotune_cache_holds_launch_options_only():
    fields = {f[0] for f in kc.Options._fields_}
    for key, e in autotune.load_cache().items():
        assert set(e["best"]) <= fields, e["best"]
        assert e["order"] in kc.ORDERS and e["k"] >= 3
    assert set(autotune.GRID) <= fields


def test_autotune_coordinate_descent_finds_the_separable_optimum():
    """On an objective that is a sum over knobs, one sweep of the coordinate
    descent reaches the grid's minimum; every evaluation is cached."""
    calls = []
    pref = {"waves_per_root": 4, "chunk": 16, "compress": 64, "compress_level": 0, "class_streams": 2}

    def cost(c):
        calls.append(dict(c))
        return 100.0 + sum(0.0 if c.get(k, 0) == v else 10.0 + abs(c.get(k, 0) - v) for k, v in pref.items())

    best, table = autotune.coordinate_descent(cost, log=lambda *a: None)
    assert best == {k: v for k, v in pref.items() if v != 0}
    assert len(calls) == len(table) == len({str(sorted(c.items())) for c in calls})
    assert min(table.values()) == 100.0


def test_saved_scheduler_model_matches_the_network():
    with open(scheduler.MODEL_PATH) as f:
        models = json.load(f)["models"]
    assert models
    for k, m in models.items():
        assert len(m["params"]) == kc.MLP_NPARAMS
        assert len(m["mean"]) == kc.MLP_IN and len(m["std"]) == kc.MLP_IN
        assert all(v > 0 for v in m["std"])
        assert np.all(np.isfinite(m["params"]))
        assert m["validation"]["mse"] < 0.1 * m["validation"]["target_var"]
    params, norm = scheduler.load_model("cpu", 8)
    assert params.numel() == kc.MLP_NPARAMS and norm.numel() == 2 * kc.MLP_IN


def test_spearman_uses_average_ranks_for_ties():
    from scipy.stats import spearmanr
    rng = np.random.default_rng(0)
    a = rng.integers(0, 5, 300).astype(float)
    b = a + rng.normal(0, 1, 300)
    assert abs(scheduler.spearman(a, b) - spearmanr(a, b).statistic) < 1e-12


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_generators_are_deterministic_and_follow_the_recipe():
    w1 = graphgen.workload(5, scale=0.001)
    w2 = graphgen.workload(5, scale=0.001)
    (rp, ci), (rp2, ci2) = w1.graphs[0], w2.graphs[0]
    assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2)
    assert oracle.validate(rp, ci)
    # the largest planted clique bounds the degeneracy from below
    core = oracle.core_numbers(rp, ci)
    assert core.max() >= max(w1.params["planted"]) - 1
    w4 = graphgen.workload(4, scale=0.03)
    assert len(w4.graphs) == len(w4.ks) and all(3 <= k <= 9 for k in w4.ks)
    for (rp, ci), (n, d, k) in zip(w4.graphs, w4.params["graphs"]):
        assert len(rp) - 1 == n and oracle.validate(rp, ci)
        assert abs(len(ci) / n - d) < 0.5 * d  # mean degree near its draw


def test_root_shares_partition_the_vertices():
    """paper_2203_13512_amd.shares assigns every vertex to exactly one of S
    shares by a multiplicative hash of its id; consecutive ids (and the
    low-id hubs of R-MAT graphs) spread over all shares."""
    torch = pytest.importorskip("torch")
    from paper_2203_13512_amd import shares
    n, S = 100_003, 16
    idx = shares.share_index(n, S, torch.device("cpu")).numpy()
    assert idx.shape == (n,) and idx.min() >= 0 and idx.max() < S
    counts = np.bincount(idx, minlength=S)
    assert counts.sum() == n and counts.min() > 0.95 * n / S and counts.max() < 1.05 * n / S
    assert len(set(idx[:64].tolist())) == S  # the first 64 ids reach every share
    assert np.array_equal(shares.share_index(n, 1, torch.device("cpu")).numpy(), np.zeros(n, dtype=np.int64))
