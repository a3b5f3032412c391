"""SDegree with the out-neighbour reduction of Sec. 7.2 (orders
'degree_reduced' and 'core_reduced'): Alg. 5 on each root's induced DAG G_u.

Counts equal the definition; per-root joins, Lemma-2 work (|C| + |L_x| per
join on G_u) and node counts equal the oracle's reduced recursion, for whole
roots and for roots split into edge tasks, with and without pruning;
per-vertex participation and the listing equal the oracle's, also for roots
of the 4096-entry list class.  Roots beyond it are refused, not
approximated.
"""
import math
import sys

import numpy as np
import pytest

import graphgen
import oracle
from tests import _graphs as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2203_13512_amd as kc  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(g):
    rp, ci = g
    return (torch.from_numpy(np.ascontiguousarray(rp, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(ci, dtype=np.int32)).cuda())


GRAPHS = [
    ("er", lambda: graphgen.erdos_renyi(400, 0.06, planted=[14, 11, 9], seed=3)),
    ("chunglu", lambda: graphgen.chung_lu(6000, 10.0, 2.1, 500.0, planted=[22, 16], seed=3)),
    ("rmat", lambda: graphgen.rmat(11, 8, 0.57, 0.19, 0.19, 6, 12, 24, 0.9, seed=3)),
    ("union", lambda: G.disjoint_union([G.complete(12), graphgen.erdos_renyi(90, 0.35, seed=3), G.complete(6)])),
    ("bipartite", lambda: G.bipartite_with_clique(200, 150, 9)),
]


@pytest.mark.parametrize("order", ["degree_reduced", "core_reduced"])
@pytest.mark.parametrize("name,make", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_reduced_sdegree_matches_oracle(order, name, make):
    g = make()
    rp, ci = dev(g)
    for k in (3, 4, 5, 7):
        want = oracle.count(*g, k)
        for kw in (dict(), dict(split=1, split_threshold=1.0), dict(split=-1, chunk=3),
                   dict(disable=kc.NO_PRUNE), dict(disable=kc.NO_PRUNE, split=1, split_threshold=1.0)):
            say("reduced", name, order, k, kw)
            total, pl, per = oracle.method_count(*g, k, order, disable=kw.get("disable", 0))
            assert total == want
            c, st = kc.count(rp, ci, k, order, root_logs=True, **kw)
            assert c == want, kw
            lg = {key: v.cpu().numpy() for key, v in st["root_logs"].items()}
            assert st["prelist_count"] == pl
            # per-vertex attribution: the cliques listed from each root (a
            # clique component's Pre-List cliques go to its smallest vertex,
            # which is no root)
            roots = per["dplus"] >= k - 1
            assert np.array_equal(lg["count"][roots], per["count"][roots].astype(np.int64)), kw
            assert int(lg["count"].sum()) == c
            assert np.array_equal(lg["isect"], per["isect"].astype(np.int64)), kw
            assert np.array_equal(lg["work"], per["work"].astype(np.int64)), kw
            assert st["nodes"] == int(per["nodes"].sum()) and st["isect"] == int(per["isect"].sum())


def test_reduction_lowers_the_logged_work():
    """On the same graph and orientation the reduced recursion performs no
    more joins and fewer Lemma-2 elements than the unreduced one."""
    g = graphgen.chung_lu(20000, 12.0, 2.1, 800.0, planted=[30, 24], seed=5)
    rp, ci = dev(g)
    for k in (4, 6):
        c0, s0 = kc.count(rp, ci, k, "degree", stats=True)
        c1, s1 = kc.count(rp, ci, k, "degree_reduced", stats=True)
        say("reduction", k, s0["isect"], s1["isect"], s0["work"], s1["work"], s0["list_ms"], s1["list_ms"])
        assert c0 == c1 == oracle.count(*g, k)
        assert s1["isect"] <= s0["isect"] and s1["work"] < s0["work"] and s1["nodes"] == s0["nodes"]


@pytest.mark.parametrize("order", ["degree_reduced", "core_reduced"])
def test_reduced_per_vertex_and_listing(order):
    """Per-vertex participation equals the oracle's; the listing is the
    oracle's set of k-cliques as sorted tuples (Sec. 3.1)."""
    for name, make in GRAPHS:
        g = make()
        rp, ci = dev(g)
        for k in (3, 4, 6):
            say("reduced per-vertex / listing", name, order, k)
            want, wpv = oracle.count(*g, k, per_vertex=True)
            for kw in (dict(), dict(split=1, split_threshold=1.0)):
                c, pv = kc.count(rp, ci, k, order, per_vertex=True, **kw)
                assert c == want and np.array_equal(pv.cpu().numpy(), wpv.astype(np.int64)), kw
            if want <= 200000:
                rows, total = kc.list_cliques(rp, ci, k, order)
                assert total == want
                got = np.sort(rows.cpu().numpy(), axis=1)
                exp, _ = oracle.list_cliques(*g, k)
                assert np.array_equal(got[np.lexsort(got.T[::-1])], np.asarray(exp, dtype=np.int32))


def _bipartite_with_clique_np(a, b, m):
    """G.bipartite_with_clique built with numpy (for sizes where a Python
    edge list is slow)."""
    left = np.repeat(np.arange(a, dtype=np.int32), b)
    right = np.tile(np.arange(a, a + b, dtype=np.int32), a)
    iu, ju = np.triu_indices(m, 1)
    clique = np.stack([iu + a, ju + a], axis=1).astype(np.int32)
    return graphgen.from_edges(a + b, np.concatenate([np.stack([left, right], axis=1), clique]))


@pytest.mark.parametrize("order", ["degree_reduced", "core_reduced"])
def test_reduced_roots_of_the_4096_entry_class(order):
    """Roots of 1025..4096 out-neighbours (the 4096-entry list class):
    K_{1100,1100} plus a 9-clique on the right.  In degree order every left
    vertex has the 1100 right vertices as out-neighbours.  Counts, per-vertex
    values, listing and per-root logs equal the oracle's."""
    g = G.bipartite_with_clique(1100, 1100, 9)
    rp, ci = dev(g)
    for k in (3, 4, 5):
        want, wpv = oracle.count(*g, k, per_vertex=True)
        total, pl, per = oracle.method_count(*g, k, order)
        assert total == want == 1100 * math.comb(9, k - 1) + math.comb(9, k)
        roots = per["dplus"] >= k - 1
        for kw in (dict(), dict(split=1, split_threshold=1.0), dict(disable=kc.NO_PRUNE)):
            say("4096-entry class", order, k, kw)
            if "disable" in kw:
                total, pl, per = oracle.method_count(*g, k, order, disable=kw["disable"])
            c, st = kc.count(rp, ci, k, order, root_logs=True, **kw)
            assert c == want, kw
            assert st["max_out_degree"] > 1024 and st["class_tasks"][3] > 0
            lg = {key: v.cpu().numpy() for key, v in st["root_logs"].items()}
            assert np.array_equal(lg["count"][roots], per["count"][roots].astype(np.int64)), kw
            assert np.array_equal(lg["isect"], per["isect"].astype(np.int64)), kw
            assert np.array_equal(lg["work"], per["work"].astype(np.int64)), kw
            assert st["nodes"] == int(per["nodes"].sum())
        c, pv = kc.count(rp, ci, k, order, per_vertex=True)
        assert c == want and np.array_equal(pv.cpu().numpy(), wpv.astype(np.int64))
        rows, t = kc.list_cliques(rp, ci, k, order)
        assert t == want
        got = np.sort(rows.cpu().numpy(), axis=1)
        exp, _ = oracle.list_cliques(*g, k)
        assert np.array_equal(got[np.lexsort(got.T[::-1])], np.asarray(exp, dtype=np.int32))


def test_reduced_dense_4096_entry_class_closed_form():
    """K_1030 minus one edge: roots of up to 1028 out-neighbours whose G_u are
    dense (the pool holds about d+^2/2 entries); C(n,k) - C(n-2,k-2)."""
    n = 1030
    big = dev(G.complete_minus_edge(n))
    for order in ("degree_reduced", "core_reduced"):
        say("K_n - e, reduced", order)
        c, st = kc.count(*big, 4, order, stats=True)
        assert c == math.comb(n, 4) - math.comb(n - 2, 2)
        assert st["class_tasks"][3] > 0


def test_reduced_roots_beyond_its_lists_are_refused():
    # out-degrees above 4096 (the 16384-entry list class): K_{4100,4100}
    # plus a 5-clique on the right, so that its roots have work
    big = dev(_bipartite_with_clique_np(4100, 4100, 5))
    with pytest.raises(kc.KCliqueError) as e:
        kc.count(*big, 4, "degree_reduced")
    assert e.value.status == kc.EUNSUPPORTED


def test_reduced_full_size_workload_2():
    """Workload 2 (Chung-Lu, 1M vertices) at k = 5: the count equals the
    oracle's golden count."""
    import json
    import os
    with open(os.path.join(G.GOLDEN, "fullsize_w2_k5_degree.json")) as f:
        gold = json.load(f)
    w = G.workload_cached(2)
    rp_h, ci_h = w.graphs[0]
    assert G.graph_sha(rp_h, ci_h) == gold["graph_sha256"]
    rp, ci = dev((rp_h, ci_h))
    c, st = kc.count(rp, ci, 5, "degree_reduced", stats=True)
    say("workload 2, k = 5, reduced SDegree:", c, "listing", round(st["list_ms"], 1), "ms; work", st["work"],
        "joins", st["isect"])
    assert c == gold["count"]
    assert st["nodes"] == gold["nodes_total"]
    assert st["work"] < gold["work_total"] and st["isect"] <= gold["isect_total"]
