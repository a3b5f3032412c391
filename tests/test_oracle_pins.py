"""Pins the CPU oracle to values fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every expected value is a
closed form, an independent brute force, or a value printed in the paper
(fixtures under tests/golden/ with their citations).
"""
import itertools
import math

import numpy as np
import pytest

import graphgen
import oracle
from tests import _graphs as G

pytestmark = pytest.mark.filterwarnings("ignore")


# ----------------------------------------------------------------- binomial
def test_binom_matches_exact_integers():
    for n in range(0, 70):
        for k in range(0, n + 2):
            exact = math.comb(n, k)
            got = oracle.binom(n, k)
            if exact < 2 ** 64:
                assert got == exact, (n, k)
            else:
                assert got is None, (n, k)


def test_binom_paper_overflow_example():
    # a 201-clique holds about 1.8e27 20-cliques (experimental setup)
    exp = G.paper_expected()
    assert exp["binom_201_20_overflows"] == ["1"]
    assert math.comb(201, 20) > 2 ** 64
    assert 1.79e27 < math.comb(201, 20) < 1.80e27
    assert oracle.binom(201, 20) is None
    assert oracle.binom(67, 33) == math.comb(67, 33)  # largest fitting central binomial
    assert oracle.binom(68, 34) is None


# ------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 24])
def test_complete_graph_counts(n):
    rp, ci = G.complete(n)
    for k in range(1, n + 2):
        c, pv = oracle.count(rp, ci, k, per_vertex=True)
        assert c == math.comb(n, k)
        assert all(int(x) == math.comb(n - 1, k - 1) for x in pv)
        if n <= 24:
            cb = oracle.count_brute(rp, ci, k)
            assert cb == math.comb(n, k)


@pytest.mark.parametrize("parts", [(1, 1, 1), (2, 3), (3, 1, 4, 1, 5), (2, 2, 2, 2, 2, 2), (7, 1, 3, 6)])
def test_complete_multipartite_counts(parts):
    (rp, ci), owner = G.multipartite(parts)
    for k in range(1, len(parts) + 2):
        c, pv = oracle.count(rp, ci, k, per_vertex=True)
        assert c == G.elementary_symmetric(parts, k)
        for v in range(len(owner)):
            rest = [a for j, a in enumerate(parts) if j != owner[v]]
            assert int(pv[v]) == G.elementary_symmetric(rest, k - 1)


def test_disjoint_union_is_additive():
    parts = [G.complete(6), G.multipartite((2, 3, 2))[0], graphgen.erdos_renyi(40, 0.3, seed=7)]
    rp, ci = G.disjoint_union(parts)
    for k in range(1, 6):
        total = sum(oracle.count(a, b, k) for a, b in parts)
        assert oracle.count(rp, ci, k) == total


# ------------------------------------------------------------- brute force
def test_all_graphs_on_six_vertices():
    """Every labelled graph on 6 vertices: brute force == ordered recursion,
    and per-vertex sums equal k times the count."""
    n = 6
    for mask in range(1 << 15):
        rp, ci = G.graph_from_mask(n, mask)
        for k in range(1, 7):
            cb, pb = oracle.count_brute(rp, ci, k, per_vertex=True)
            co, po = oracle.count(rp, ci, k, per_vertex=True)
            assert cb == co, (mask, k)
            assert np.array_equal(pb, po), (mask, k)
            assert int(po.sum()) == k * co


def test_python_brute_force_on_sampled_small_graphs():
    rng = np.random.default_rng(11)
    for trial in range(60):
        n = int(rng.integers(1, 12))
        p = float(rng.uniform(0.1, 0.95))
        rp, ci = graphgen.erdos_renyi(n, p, seed=int(rng.integers(1 << 30)))
        for k in range(1, 6):
            c_py, pv_py = G.py_brute_count(rp, ci, k)
            c0, pv0 = oracle.count_brute(rp, ci, k, per_vertex=True)
            c1, pv1 = oracle.count(rp, ci, k, per_vertex=True)
            assert c_py == c0 == c1
            assert list(map(int, pv0)) == pv_py == list(map(int, pv1))


def test_vertex_count_matches_per_vertex():
    rp, ci = graphgen.erdos_renyi(120, 0.2, planted=[9, 7], seed=5)
    for k in (2, 3, 4, 5):
        _, pv = oracle.count(rp, ci, k, per_vertex=True)
        for v in range(0, 120, 7):
            assert oracle.vertex_count(rp, ci, k, v) == int(pv[v])
    assert oracle.vertex_count(rp, ci, 4, 3, budget=1) is None


def test_roots_subset_partitions_the_count():
    rp, ci = graphgen.erdos_renyi(200, 0.1, planted=[10], seed=9)
    total = oracle.count(rp, ci, 4)
    a = oracle.count_roots(rp, ci, 4, np.arange(0, 77))
    b = oracle.count_roots(rp, ci, 4, np.arange(77, 200))
    assert a[2] and b[2]
    assert a[0] + b[0] == total


# ------------------------------------------------------- paper's examples
def test_paper_example_counts():
    exp = G.paper_expected()
    (rp, ci), n = G.paper_example_graph()
    assert oracle.validate(rp, ci)
    assert oracle.count(rp, ci, 4) == int(exp["count_k4_G"][0])
    assert oracle.count_brute(rp, ci, 4) == 3


def test_paper_precore_example():
    exp = G.paper_expected()
    (rp, ci), n = G.paper_example_graph()
    removed = oracle.precore(rp, ci, 4)
    assert sorted(int(v) + 1 for v in np.nonzero(removed)[0]) == [int(x) for x in exp["precore_k4_removed"]]


def test_paper_prelist_example():
    exp = G.paper_expected()
    (rp, ci), n = G.paper_example_graph()
    removed = oracle.precore(rp, ci, 4)
    after, cnt, pv, ncomp = oracle.prelist(rp, ci, 4, removed, per_vertex=True)
    assert cnt == int(exp["prelist_k4_count"][0])
    newly = sorted(int(v) + 1 for v in np.nonzero(after & ~removed)[0])
    assert newly == [int(x) for x in exp["prelist_k4_removed"]]
    assert ncomp == 1
    assert [int(pv[v - 1]) for v in newly] == [1, 1, 1, 1]


def _reduced_example():
    (rp, ci), n = G.paper_example_graph()
    removed = oracle.precore(rp, ci, 4)
    after, _, _, _ = oracle.prelist(rp, ci, 4, removed)
    return rp, ci, after


def test_paper_sdegree_example_trace():
    """Example 4: degree DAG of the reduced graph, roots v2 and v5, and the
    recursion from v2 (which expands only v3 and v4)."""
    exp = G.paper_expected()
    rp, ci, removed = _reduced_example()
    drp, dci = oracle.degree_dag(rp, ci, removed)
    dplus = np.diff(drp)
    roots = sorted(int(v) + 1 for v in range(12) if dplus[v] >= 3)
    assert roots == [int(x) for x in exp["sdegree_k4_roots"]]
    # out-neighbour sets (0-based), hand-derived from the (degree, id) order
    nplus = {u + 1: sorted(int(x) + 1 for x in dci[drp[u]:drp[u + 1]]) for u in range(6)}
    assert nplus == {1: [], 2: [1, 3, 4, 6], 3: [1, 4], 4: [1, 6], 5: [1, 3, 6], 6: [1]}
    total, per = oracle.sdegree_dag(drp, dci, 4)
    assert total == 2
    assert int(per["count"][1]) == int(exp["sdegree_k4_cliques_from_v2"][0])
    assert int(per["count"][4]) == 0
    # from v2: the top call, then v3 and v4 expand (v1 and v6 are pruned by
    # d+ <= l-2); each expansion does one join at l = 2 -> 3 calls, 4 joins
    assert int(per["nodes"][1]) == 3 and int(per["isect"][1]) == 4
    # |C| + d+ summed: top joins (4+2) + (4+2); then (2+2) and (2+1)
    assert int(per["elems"][1]) == 6 + 6 + 4 + 3
    # from v5: one join (v3), |C'| = 1 is not > l-2 = 1, so no recursion
    assert int(per["nodes"][4]) == 1 and int(per["isect"][4]) == 1
    # the full SDegree pipeline gives the same plus the Pre-List clique
    (grp, gci), _ = G.paper_example_graph()
    t, pl, _ = oracle.method_count(grp, gci, 4, "degree")
    assert (t, pl) == (3, 1)


def test_paper_merge_join_example():
    exp = G.paper_expected()
    a = [int(x) for x in exp["merge_a"]]
    b = [int(x) for x in exp["merge_b"]]
    assert list(oracle.merge_join(a, b)) == [int(x) for x in exp["merge_result"]]
    rng = np.random.default_rng(3)
    for _ in range(200):
        x = np.unique(rng.integers(0, 300, rng.integers(0, 80)))
        y = np.unique(rng.integers(0, 300, rng.integers(0, 80)))
        assert list(oracle.merge_join(x, y)) == sorted(set(x.tolist()) & set(y.tolist()))


def _example_local_graph():
    """Induced subgraph on v1..v6 (local index = vertex name - 1)."""
    (rp, ci), n = G.paper_example_graph()
    adj = np.zeros((6, 6), dtype=np.uint8)
    for u in range(6):
        for w in ci[rp[u]:rp[u + 1]]:
            if w < 6:
                adj[u, w] = 1
    return adj


def test_paper_coloring_example():
    exp = G.paper_expected()
    adj = _example_local_graph()
    order, color = oracle.greedy_color(adj, np.arange(1, 7))
    assert [int(v) + 1 for v in order] == [int(x) for x in exp["color_order"]]
    assert int(color[3]) == int(exp["color_v4"][0])
    # proper coloring
    for u in range(6):
        for w in range(6):
            if adj[u, w]:
                assert color[u] != color[w]


def test_paper_bitmap_table():
    exp = G.paper_expected()
    adj = _example_local_graph()
    color, B = oracle.bitcol_encode(adj, np.arange(1, 7), 3)
    want = [tuple(int(t) for t in cell.split(",")) for cell in exp["table3_B"]]
    assert [tuple(int(x) for x in row) for row in B] == want
    joined = B[2] & B[3]
    assert tuple(int(x) for x in joined) == tuple(int(t) for t in exp["bitjoin_v3_v4"][0].split(","))
    # decode <3,0> with L = 3: bits 0 and 1 of word 0 -> v1, v2
    members = [j * 3 + i + 1 for j in range(2) for i in range(3) if (int(joined[j]) >> i) & 1]
    assert members == [1, 2]


# ------------------------------------------------------ preprocessing pins
def _py_core_numbers(rp, ci):
    """Core numbers from the definition: largest c such that v survives
    repeated deletion of vertices of degree < c."""
    n = len(rp) - 1
    core = [0] * n
    c = 0
    while True:
        alive = set(range(n))
        changed = True
        while changed:
            changed = False
            for v in list(alive):
                if sum(1 for w in ci[rp[v]:rp[v + 1]] if int(w) in alive) < c:
                    alive.discard(v)
                    changed = True
        if not alive:
            break
        for v in alive:
            core[v] = c
        c += 1
    return core


def test_core_numbers_from_definition():
    rng = np.random.default_rng(2)
    for t in range(25):
        n = int(rng.integers(2, 45))
        rp, ci = graphgen.erdos_renyi(n, float(rng.uniform(0.05, 0.6)), planted=[int(rng.integers(2, 8))],
                                      seed=int(rng.integers(1 << 30)))
        assert list(map(int, oracle.core_numbers(rp, ci))) == _py_core_numbers(rp, ci)


def test_precore_is_the_k_minus_1_core():
    rng = np.random.default_rng(4)
    for t in range(20):
        rp, ci = graphgen.chung_lu(3000, 8.0, 2.2, 200.0, planted=[10, 6], seed=int(rng.integers(1 << 30)))
        core = oracle.core_numbers(rp, ci)
        for k in (3, 4, 6, 9):
            removed = oracle.precore(rp, ci, k)
            assert np.array_equal(removed.astype(bool), core < k - 1)


def test_prelist_on_unions_of_cliques():
    parts = [G.complete(s) for s in (3, 5, 8)] + [G.multipartite((2, 2, 3))[0]]
    rp, ci = G.disjoint_union(parts)
    for k in (3, 4, 5):
        removed = oracle.precore(rp, ci, k)
        after, cnt, pv, ncomp = oracle.prelist(rp, ci, k, removed, per_vertex=True)
        expected = sum(math.comb(s, k) for s in (3, 5, 8))
        assert cnt == expected
        # K_s survives Pre-Core (degrees s-1 >= k-1) exactly when s >= k
        assert ncomp == sum(1 for s in (3, 5, 8) if s >= k)
        # the multipartite component is never a clique and stays
        assert not after[-7:].any()


def test_degeneracy_dag_properties():
    rng = np.random.default_rng(8)
    for t in range(10):
        rp, ci = graphgen.chung_lu(4000, 10.0, 2.1, 300.0, planted=[15], seed=int(rng.integers(1 << 30)))
        n = len(rp) - 1
        removed = np.zeros(n, dtype=np.uint8)
        drp, dci, rnd, core = oracle.degeneracy_dag(rp, ci, removed)
        # the peel's levels are the core numbers
        assert np.array_equal(core, oracle.core_numbers(rp, ci))
        # out-degree never exceeds the core number (degeneracy bound)
        assert np.all(np.diff(drp) <= core)
        # every edge appears exactly once, oriented by (round, id)
        assert drp[-1] * 2 == len(ci)
        for u in range(0, n, 97):
            for v in dci[drp[u]:drp[u + 1]]:
                assert (rnd[u], u) < (rnd[v], v)


# --------------------------------------------------------- method results
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_methods_equal_definition(seed):
    """SDegree and BitCol as the paper orders them (Pre-Core, Pre-List,
    orientation, listing) reach the plain count (Theorem 1)."""
    rng = np.random.default_rng(seed)
    graphs = [
        graphgen.erdos_renyi(300, 0.08, planted=[12, 9, 7], seed=seed),
        graphgen.chung_lu(3000, 12.0, 2.1, 400.0, planted=[14, 10], seed=seed),
        graphgen.rmat(10, 8, 0.57, 0.19, 0.19, 6, 10, 20, 0.9, seed=seed),
        G.disjoint_union([G.complete(9), graphgen.erdos_renyi(60, 0.4, seed=seed), G.complete(5)]),
    ]
    for rp, ci in graphs:
        for k in (3, 4, 5, 6):
            want = oracle.count(rp, ci, k)
            sd, _, per_s = oracle.method_count(rp, ci, k, "degree")
            bc, _, per_b = oracle.method_count(rp, ci, k, "color")
            assert sd == want and bc == want, (k, sd, bc, want)
            for L in (3, 24):
                assert oracle.method_count(rp, ci, k, "color", L=L)[0] == want
            # BitCol's per-root words = joins x ceil(s/32)
            s = per_b["dplus"].astype(np.int64)
            assert np.array_equal(per_b["work"], per_b["isect"] * ((s + 31) // 32))
            # Lemma 4: cost of the recursion from u is at most
            # 2 D (k + (k-1)/2) (D/2)^(k-3) d+_u, with D the max out-degree
            D = float(max(1, per_s["dplus"].max()))
            bound = 2 * D * (k + (k - 1) / 2) * (D / 2) ** (k - 3) * per_s["dplus"].astype(float)
            assert np.all(per_s["work"].astype(float) <= bound + 1e-6)


def test_k3_roots_count_oriented_triangles():
    rp, ci = graphgen.chung_lu(2000, 10.0, 2.2, 150.0, seed=12)
    n = len(rp) - 1
    removed = oracle.precore(rp, ci, 3)
    removed, pl, _, _ = oracle.prelist(rp, ci, 3, removed)
    drp, dci = oracle.degree_dag(rp, ci, removed)
    _, per = oracle.sdegree_dag(drp, dci, 3)
    for u in range(0, n, 13):
        out = set(int(x) for x in dci[drp[u]:drp[u + 1]])
        t = sum(len(out & set(int(x) for x in dci[drp[v]:drp[v + 1]])) for v in out)
        assert int(per["count"][u]) == t


def test_validate_rejects_bad_csr():
    rp, ci = G.complete(4)
    assert oracle.validate(rp, ci)
    bad = ci.copy()
    bad[0], bad[1] = bad[1], bad[0]
    assert not oracle.validate(rp, bad)  # unsorted row
    asym = graphgen.from_edges(3, [(0, 1)])
    a_rp, a_ci = asym[0].copy(), asym[1].copy()
    a_ci[0] = 2  # 0 -> 2 without 2 -> 0
    assert not oracle.validate(a_rp, a_ci)


def test_bitcol_roots_matches_the_whole_dag_run():
    """The per-root entry point (used for sampled checks on large graphs)
    returns exactly the whole-DAG run's per-root values."""
    g = graphgen.chung_lu(3000, 12.0, 2.1, 300.0, planted=[18, 12], seed=5)
    for k in (4, 6):
        rem = oracle.precore(*g, k)
        rem, _, _, _ = oracle.prelist(*g, k, rem)
        drp, dci, _, _ = oracle.degeneracy_dag(*g, rem)
        total, per = oracle.bitcol_dag(drp, dci, k)
        roots = np.flatnonzero(np.diff(drp) >= k - 1)[::3]
        sub = oracle.bitcol_roots(drp, dci, k, roots)
        for key in ("count", "nodes", "isect", "words"):
            assert np.array_equal(sub[key], per[key][roots]), key
        assert total == int(per["count"].sum())


def test_timed_bitcol_sample_counts_what_the_roots_list():
    """The time-bounded runs from a list of roots (the CPU baseline's sample;
    BitCol and SDegree) count exactly the cliques of those roots when they
    have time to finish,
    and, with all roots, the definition's count minus Pre-List's; a deadline
    that has passed stops it after the root in progress."""
    g = graphgen.chung_lu(3000, 12.0, 2.1, 300.0, planted=[18, 12], seed=5)
    k = 5
    rem = oracle.precore(*g, k)
    rem, pl, _, _ = oracle.prelist(*g, k, rem)
    drp, dci, _, _ = oracle.degeneracy_dag(*g, rem)
    roots = np.flatnonzero(np.diff(drp) >= k - 1)
    c, done, finished = oracle.bitcol_count_roots(drp, dci, k, roots, 600.0)
    assert finished and done == len(roots)
    assert c + pl == oracle.count(*g, k)
    some = roots[1::4]
    c, done, finished = oracle.bitcol_count_roots(drp, dci, k, some, 600.0)
    assert c == int(oracle.bitcol_roots(drp, dci, k, some)["count"].sum())
    c, done, finished = oracle.bitcol_count_roots(drp, dci, k, roots, 1e-9)
    assert not finished and done == 1
    ddrp, ddci = oracle.degree_dag(*g, rem)
    droots = np.flatnonzero(np.diff(ddrp) >= k - 1)
    c, done, finished = oracle.sdegree_count_roots(ddrp, ddci, k, droots, 600.0)
    assert finished and done == len(droots) and c + pl == oracle.count(*g, k)
    c, done, finished = oracle.sdegree_count_roots(ddrp, ddci, k, droots, 1e-9)
    assert not finished and done == 1
    c, done, finished = oracle.sdegree_count_roots(ddrp, ddci, k, droots, 600.0, reduce=True)
    assert finished and c + pl == oracle.count(*g, k)


def test_paper_bitcol_trace_on_the_encoded_example():
    """BitColList (Alg. 6) traced by hand on the local graph of Example 6 and
    Table 3, taken as G_u of one root u.

    DAG: u = 0 points to v1..v6 (ids 1..6) and the 12 edges of the local graph
    point from the smaller to the larger id, so G_u is exactly that graph and
    its greedy coloring is Example 6's: colors (v1..v6) = (1, 2, 3, 4, 2, 3),
    B(v1..v6) = {}, {v1}, {v1,v2}, {v1,v2,v3,v6}, {v1}, {v1,v2,v5} (Table 3).

    k = 4 (top call l = 3, C = all six): v1, v2, v5 fail color >= 3.
      v3: C' = {v1,v2,v5} (join 1), l = 2: v2 -> |{v1}| = 1 (join 2),
          v5 -> 1 (join 3)                                    -> 2 cliques
      v4: C' = {v1,v2,v3,v6} (join 4), l = 2: v2 -> 1 (join 5),
          v3 -> |{v1,v2}| = 2 (join 6), v6 -> |{v1,v2}| = 2 (join 7) -> 5
      v6: C' = {v1,v2,v5} (join 8), l = 2: v2 -> 1 (join 9), v5 -> 1 (join 10)
                                                              -> 2
      9 cliques (the 9 triangles of the local graph), 10 joins, 4 calls.
    k = 5 (l = 4): only v4 has color >= 4 (the color prune of Sec. 7.1).
      v4: C' = {v1,v2,v3,v6} (join 1), l = 3: v3 -> {v1,v2} (join 2),
          l = 2: v2 -> 1 (join 3); v6 -> {v1,v2} (join 4), l = 2: v2 -> 1
          (join 5).  2 cliques, 5 joins, 4 calls.
    k = 3 (l = 2): every vertex of color >= 2 joins once with C:
      1 + 3 + 4 + 1 + 3 = 12 cliques (the 12 edges), 5 joins, 1 call.
    k = 6 (l = 5): no vertex has color >= 5: 0 cliques, 0 joins, 1 call.
    Words: one 32-bit word per join (6 local vertices).  Features of u:
    4 colors, |E_u| = 12.
    """
    exp = G.paper_expected()
    local = [(1, 2), (1, 3), (1, 4), (1, 5), (1, 6), (2, 3), (2, 4), (2, 6), (3, 4), (3, 5), (4, 6), (5, 6)]
    n = 7
    out = {v: [] for v in range(n)}
    out[0] = [1, 2, 3, 4, 5, 6]
    for a, b in local:
        out[a].append(b)
    drp = np.zeros(n + 1, dtype=np.int32)
    drp[1:] = np.cumsum([len(out[v]) for v in range(n)])
    dci = np.asarray([w for v in range(n) for w in sorted(out[v])], dtype=np.int32)
    # the coloring the trace assumes is the paper's
    colors, _ = oracle.bitcol_encode(_example_local_graph(), np.arange(1, 7), 3)
    assert [int(c) for c in colors] == [1, 2, 3, 4, 2, 3]
    assert int(colors[3]) == int(exp["color_v4"][0])
    want = {3: (12, 5, 1), 4: (9, 10, 4), 5: (2, 5, 4), 6: (0, 0, 1)}
    for k, (cnt, joins, calls) in want.items():
        total, per = oracle.bitcol_dag(drp, dci, k)
        assert int(per["count"][0]) == cnt, k
        assert int(per["isect"][0]) == joins, k
        assert int(per["nodes"][0]) == calls, k
        assert int(per["words"][0]) == joins, k
        assert int(per["colors"][0]) == 4 and int(per["edges"][0]) == 12, k
        sub = oracle.bitcol_roots(drp, dci, k, [0])
        assert [int(sub[key][0]) for key in ("count", "isect", "nodes", "words")] == [cnt, joins, calls, joins]


def test_sdegree_roots_matches_the_whole_dag_run():
    """The per-root SDegree entry point (used for sliced runs on large graphs)
    returns exactly the whole-DAG run's per-root values."""
    g = graphgen.chung_lu(3000, 12.0, 2.1, 300.0, planted=[18, 12], seed=6)
    for k in (4, 6):
        rem = oracle.precore(*g, k)
        rem, _, _, _ = oracle.prelist(*g, k, rem)
        drp, dci = oracle.degree_dag(*g, rem)
        total, per = oracle.sdegree_dag(drp, dci, k)
        roots = np.flatnonzero(np.diff(drp) >= k - 1)[::2]
        sub = oracle.sdegree_roots(drp, dci, k, roots)
        for key in ("count", "nodes", "isect", "elems"):
            assert np.array_equal(sub[key], per[key][roots]), key


@pytest.mark.parametrize("n,a,b", [(9, 0, 1), (14, 2, 5), (20, 19, 3)])
def test_complete_minus_edge_closed_form(n, a, b):
    """K_n without one edge: C(n,k) - C(n-2,k-2) cliques; its endpoints lie in
    C(n-2,k-1), every other vertex in C(n-1,k-1) - C(n-3,k-3); the methods as
    the paper orders them reach the same."""
    rp, ci = G.complete_minus_edge(n, a, b)
    for k in range(3, n + 1):
        want = math.comb(n, k) - math.comb(n - 2, k - 2)
        c, pv = oracle.count(rp, ci, k, per_vertex=True)
        assert c == want
        for v in range(n):
            exp = math.comb(n - 2, k - 1) if v in (a, b) else math.comb(n - 1, k - 1) - math.comb(n - 3, k - 3)
            assert int(pv[v]) == exp
        for method in ("degree", "color"):
            assert oracle.method_count(rp, ci, k, method)[0] == want


@pytest.mark.parametrize("r", [3, 6, 9])
def test_cocktail_party_closed_form(r):
    rp, ci = G.cocktail_party(r)
    for k in range(1, r + 2):
        c, pv = oracle.count(rp, ci, k, per_vertex=True)
        assert c == 2 ** k * math.comb(r, k)
        assert all(int(x) == 2 ** (k - 1) * math.comb(r - 1, k - 1) for x in pv)
        if k >= 3:
            for method in ("degree", "color"):
                assert oracle.method_count(rp, ci, k, method)[0] == c


@pytest.mark.parametrize("a,b,m", [(7, 6, 4), (9, 5, 5), (40, 40, 8)])
def test_bipartite_with_clique_closed_form(a, b, m):
    """K_{a,b} plus an m-clique on the right side: a C(m,k-1) + C(m,k)
    k-cliques for k >= 3 (brute force on the small ones)."""
    rp, ci = G.bipartite_with_clique(a, b, m)
    for k in range(3, m + 2):
        c, pv = oracle.count(rp, ci, k, per_vertex=True)
        assert c == a * math.comb(m, k - 1) + math.comb(m, k)
        want_pv = [math.comb(m, k - 1)] * a + [a * math.comb(m - 1, k - 2) + math.comb(m - 1, k - 1)] * m
        assert [int(x) for x in pv] == want_pv + [0] * (b - m)
        if a + b <= 16:
            assert G.py_brute_count(rp, ci, k)[0] == c
        for method in ("degree", "color", "core"):
            assert oracle.method_count(rp, ci, k, method)[0] == c


def test_listing_matches_brute_force():
    """The oracle's listing (Sec. 3.1) writes exactly the k-subsets that are
    cliques, each once, as ascending ids in lexicographic order."""
    rng = np.random.default_rng(13)
    for trial in range(40):
        n = int(rng.integers(1, 13))
        rp, ci = graphgen.erdos_renyi(n, float(rng.uniform(0.2, 0.95)), seed=int(rng.integers(1 << 30)))
        adj = [set(int(x) for x in ci[rp[v]:rp[v + 1]]) for v in range(n)]
        for k in range(1, 7):
            want = [S for S in itertools.combinations(range(n), k)
                    if all(b in adj[a] for a, b in itertools.combinations(S, 2))]
            rows, total = oracle.list_cliques(rp, ci, k)
            assert total == len(want)
            assert [tuple(int(x) for x in r) for r in rows] == want
            if total > 1:  # a bounded buffer keeps the first rows and the full count
                part, t2 = oracle.list_cliques(rp, ci, k, capacity=total // 2)
                assert t2 == total and np.array_equal(part, rows[: total // 2])
    (rp, ci), n = G.paper_example_graph()
    rows, total = oracle.list_cliques(rp, ci, 4)
    # Example 1: {v1,v2,v3,v4}, {v1,v2,v4,v6}, {v9,v10,v11,v12} (0-based here)
    assert total == 3 and [tuple(int(x) for x in r) for r in rows] == [(0, 1, 2, 3), (0, 1, 3, 5), (8, 9, 10, 11)]


def test_reduced_sdegree_trace_on_the_encoded_example():
    """SDegree with the out-neighbour reduction (Sec. 7.2) on the graph H of
    Table 3 (edges 1-2 1-3 1-4 1-5 1-6 2-3 2-4 2-6 3-4 3-5 4-6 5-6), k = 4,
    traced by hand.  Degree order (d, id): v5 < v2 < v3 < v4 < v6 < v1, so
    N+(v2) = {v1,v3,v4,v6}, N+(v3) = {v1,v4}, N+(v4) = {v1,v6},
    N+(v5) = {v1,v3,v6}, N+(v6) = {v1}; the roots (d+ >= 3) are v2 and v5.
    Root v2, local positions v1,v3,v4,v6 = 0..3, reduced lists L0 = {},
    L1 = {0,2}, L2 = {0,3}, L3 = {0}; top call l = 3, |C| = 4:
      x=0 skipped (|L| = 0 <= 1); x=1 joins (4+2) -> {0,2}, node at l = 2:
        x=0 skipped, x=2 joins (2+2) -> {0}: 1 clique;
      x=2 joins (4+2) -> {0,3}, node at l = 2: x=0 skipped, x=3 joins
        (2+1) -> {0}: 1 clique;  x=3 skipped (|L| = 1 <= 1).
      2 cliques, 4 joins, work 6+4+6+3 = 19, 3 nodes (as without reduction).
    Root v5, positions v1,v3,v6, L0 = {}, L1 = {0} (v4 is not in N+(v5)),
    L2 = {0}: every candidate is skipped (|L| <= 1): 0 joins, 1 node.
    Without the reduction v3 keeps d+ = 2 and joins once (3+2 = 5 elements)."""
    E = [(1, 2), (1, 3), (1, 4), (1, 5), (1, 6), (2, 3), (2, 4), (2, 6), (3, 4), (3, 5), (4, 6), (5, 6)]
    g = G.csr(6, [(a - 1, b - 1) for a, b in E])
    want = {"count": [0, 2, 0, 0, 0, 0], "isect": [0, 4, 0, 0, 0, 0], "work": [0, 19, 0, 0, 0, 0],
            "nodes": [0, 3, 0, 0, 1, 0]}
    c, pl, per = oracle.method_count(*g, 4, "degree_reduced")
    assert c == 2 and pl == 0
    for key, v in want.items():
        assert [int(x) for x in per[key]] == v, key
    c, pl, per = oracle.method_count(*g, 4, "degree")
    assert [int(x) for x in per["isect"]] == [0, 4, 0, 0, 1, 0]
    assert [int(x) for x in per["work"]] == [0, 19, 0, 0, 5, 0]


def test_reduced_sdegree_never_joins_more():
    """The reduction only shortens out-lists (L_x is N+(x) restricted to
    N+(u)): per root, the same nodes, no more joins and no more Lemma-2
    elements than without it; the counts agree root by root."""
    g = graphgen.chung_lu(3000, 12.0, 2.1, 300.0, planted=[18, 12], seed=9)
    for k in (3, 4, 5, 6):
        a = oracle.method_count(*g, k, "degree")[2]
        b = oracle.method_count(*g, k, "degree_reduced")[2]
        assert np.array_equal(a["count"], b["count"]) and np.array_equal(a["nodes"], b["nodes"])
        assert np.all(b["isect"] <= a["isect"]) and np.all(b["work"] <= a["work"])
        assert b["work"].sum() < a["work"].sum()
        rem = oracle.precore(*g, k)
        rem, _, _, _ = oracle.prelist(*g, k, rem)
        drp, dci = oracle.degree_dag(*g, rem)
        roots = np.flatnonzero(np.diff(drp) >= k - 1)[::5]
        sub = oracle.sdegree_roots(drp, dci, k, roots, reduce=True)
        for key, kk in (("count", "count"), ("isect", "isect"), ("elems", "work"), ("nodes", "nodes")):
            assert np.array_equal(sub[key], b[kk][roots]), key


@pytest.mark.parametrize("seed", [1, 2])
def test_ablations_and_orders_reach_the_definition(seed):
    """SDegree on the degree or the degeneracy order (Sec. 6.2: any order
    works) and BitCol reach the plain count with or without Pre-Core,
    Pre-List and pruning (preprocessing and pruning remove only nodes that
    hold no clique, Sec. 5 and Lemma 3); dropping them never lowers the
    number of joins; the degeneracy order bounds out-degrees by core numbers."""
    graphs = [
        graphgen.chung_lu(2500, 10.0, 2.1, 300.0, planted=[13, 9], seed=seed),
        G.disjoint_union([G.complete(8), graphgen.erdos_renyi(70, 0.35, seed=seed), G.complete(5)]),
    ]
    for rp, ci in graphs:
        core = oracle.core_numbers(rp, ci)
        for k in (3, 4, 5):
            want = oracle.count(rp, ci, k)
            for method in ("degree", "core", "color", "degree_reduced", "core_reduced"):
                base = oracle.method_count(rp, ci, k, method)
                assert base[0] == want
                for disable in (1, 2, 4, 7):
                    got = oracle.method_count(rp, ci, k, method, disable=disable)
                    assert got[0] == want, (method, disable)
                    if disable & 4:
                        assert got[2]["isect"].sum() >= base[2]["isect"].sum()
                if method in ("core", "core_reduced"):
                    d = base[2]["dplus"]
                    assert np.all(d <= np.maximum(core, 0))


@pytest.mark.parametrize("method", ["degree", "color", "core", "degree_reduced"])
def test_per_root_counts_partition_the_cliques(method):
    """Theorem 1: every k-clique has one root, so the oracle's per-root
    counts plus Pre-List's C(n_c, k) per clique component sum to the
    definition's count, and the cliques of a root all contain it (a root's
    count is at most its brute-force participation)."""
    g = G.disjoint_union([G.complete(9), graphgen.erdos_renyi(40, 0.45, seed=11), G.complete(6)])
    for k in (3, 4, 5):
        want, pv = oracle.count(*g, k, per_vertex=True)
        total, pl, per = oracle.method_count(*g, k, method)
        roots = per["dplus"] >= k - 1
        # the two clique components, removed by Pre-List
        assert pl == math.comb(9, k) + math.comb(6, k)
        assert total == want == int(per["count"][roots].astype(np.uint64).sum()) + pl
        assert np.all(per["count"][roots].astype(np.int64) <= pv[roots].astype(np.int64))
