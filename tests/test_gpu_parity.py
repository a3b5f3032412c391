"""GPU parity: the HIP library against the CPU oracle, bit for bit.

Every test calls the library through its C interface (the binding only
marshals arguments) and compares with the oracle on the same seeded inputs.
Counts and per-vertex participation are unique, so they must be identical;
the per-root work logs and features are fixed by the orientation, coloring
and pruning readings both sides implement, so they must be identical too.
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


def gcount(g, k, order, **kw):
    rp, ci = dev(g)
    return kc.count(rp, ci, k, order, **kw)


def gpv(g, k, order, **kw):
    rp, ci = dev(g)
    c, pv = kc.count(rp, ci, k, order, per_vertex=True, **kw)
    return c, pv.cpu().numpy()


ORDERS = ["degree", "color"]


# ------------------------------------------------------------- small cases
@pytest.mark.parametrize("order", ORDERS)
def test_paper_example(order):
    (rp, ci), n = G.paper_example_graph()
    for k in range(1, 7):
        say("paper example", order, k)
        want, wpv = oracle.count(rp, ci, k, per_vertex=True)
        assert gcount((rp, ci), k, order) == want
        c, pv = gpv((rp, ci), k, order)
        assert c == want and np.array_equal(pv, wpv.astype(np.int64))
    assert gcount((rp, ci), 4, order) == 3


@pytest.mark.parametrize("order", ORDERS)
def test_edge_cases(order):
    say("edge cases", order)
    empty = (np.zeros(1, np.int32), np.zeros(0, np.int32))
    for k in (1, 2, 3, 5):
        assert kc.count(*empty, k, order) == 0
    iso = (np.zeros(6, np.int32), np.zeros(0, np.int32))  # 5 isolated vertices
    assert kc.count(*iso, 1, order) == 5
    assert kc.count(*iso, 2, order) == 0
    assert kc.count(*iso, 3, order) == 0
    k4 = G.complete(4)
    assert kc.count(*k4, 5, order) == 0  # k > n
    assert kc.count(*k4, 4, order) == 1
    assert kc.count(*k4, 2, order) == 6
    c, pv = kc.count(*k4, 1, order, per_vertex=True)
    assert c == 4 and list(pv) == [1, 1, 1, 1]
    c, pv = kc.count(*k4, 2, order, per_vertex=True)
    assert c == 6 and list(pv) == [3, 3, 3, 3]
    for bad_k in (0, -3):
        with pytest.raises(kc.KCliqueError) as e:
            kc.count(*k4, bad_k, order)
        assert e.value.status == kc.EINVAL


@pytest.mark.parametrize("order", ORDERS)
def test_malformed_graphs_are_rejected(order):
    say("malformed", order)
    rp, ci = G.complete(5)
    bad = ci.copy()
    bad[0], bad[1] = bad[1], bad[0]  # unsorted row
    asym_rp, asym_ci = graphgen.from_edges(3, [(0, 1)])
    asym_ci = asym_ci.copy()
    asym_ci[0] = 2  # 0 -> 2 without 2 -> 0
    loop = (np.array([0, 1, 2], np.int32), np.array([0, 0], np.int32))  # self-loop
    outr = (np.array([0, 1, 2], np.int32), np.array([1, 7], np.int32))  # id out of range
    for g in [(rp, bad), (asym_rp, asym_ci), loop, outr]:
        for on_gpu in (False, True):
            with pytest.raises(kc.KCliqueError) as e:
                if on_gpu:
                    gcount(g, 3, order)
                else:
                    kc.count(*g, 3, order)
            assert e.value.status == kc.EINVAL


@pytest.mark.parametrize("order", ORDERS)
def test_overflow_is_reported(order):
    """A 201-clique holds about 1.8e27 20-cliques (more than 2^64): Pre-List
    meets it as an isolated clique component and must report the overflow."""
    say("overflow K201 k=20", order)
    g = G.complete(201)
    with pytest.raises(kc.KCliqueError) as e:
        gcount(g, 20, order)
    assert e.value.status == kc.EOVERFLOW
    # the same component at k = 8 fits
    assert gcount(g, 8, order) == math.comb(201, 8)


@pytest.mark.parametrize("order", ORDERS)
def test_closed_forms(order):
    for n in (3, 7, 33, 70):
        g = G.complete(n)
        for k in (3, 4, 6):
            say("complete", n, k, order)
            c, pv = gpv(g, k, order)
            assert c == math.comb(n, k)
            assert np.all(pv == math.comb(n - 1, k - 1))
    for parts in [(3, 1, 4, 1, 5, 9, 2, 6), (2,) * 12, (30, 20, 10, 5)]:
        (rp, ci), owner = G.multipartite(parts)
        for k in (3, 4, 5):
            say("multipartite", parts, k, order)
            c, pv = gpv((rp, ci), k, order)
            assert c == G.elementary_symmetric(parts, k)
            for v in range(len(owner)):
                rest = [a for j, a in enumerate(parts) if j != owner[v]]
                assert int(pv[v]) == G.elementary_symmetric(rest, k - 1)
    # a union of cliques is removed entirely by Pre-List
    g = G.disjoint_union([G.complete(s) for s in (4, 9, 17)])
    for k in (3, 4, 9):
        say("clique union", k, order)
        assert gcount(g, k, order) == sum(math.comb(s, k) for s in (4, 9, 17))


def _random_graphs(seed):
    return [
        ("er", graphgen.erdos_renyi(400, 0.06, planted=[14, 11, 9], seed=seed)),
        ("chunglu", graphgen.chung_lu(6000, 10.0, 2.1, 500.0, planted=[22, 16], seed=seed)),
        ("rmat", graphgen.rmat(11, 8, 0.57, 0.19, 0.19, 6, 12, 24, 0.9, seed=seed)),
        ("union", G.disjoint_union([G.complete(12), graphgen.erdos_renyi(90, 0.35, seed=seed), G.complete(6)])),
    ]


@pytest.mark.parametrize("seed", [1, 2])
@pytest.mark.parametrize("order", ORDERS)
def test_random_graphs_counts_and_per_vertex(seed, order):
    for name, g in _random_graphs(seed):
        for k in (3, 4, 5, 6, 8):
            say("random", name, seed, order, k)
            want, wpv = oracle.count(*g, k, per_vertex=True)
            c, pv = gpv(g, k, order)
            assert c == want, (name, k)
            assert np.array_equal(pv, wpv.astype(np.int64)), (name, k)
            assert int(pv.sum()) == k * c
            assert gcount(g, k, order) == want


@pytest.mark.parametrize("order", ORDERS)
def test_host_entry_points(order):
    g = graphgen.chung_lu(3000, 9.0, 2.2, 300.0, planted=[15], seed=3)
    for k in (3, 5, 7):
        say("host entry points", order, k)
        want, wpv = oracle.count(*g, k, per_vertex=True)
        assert kc.count_host(*g, k, order) == want
        c, pv = kc.per_vertex_host(*g, k, order)
        assert c == want and np.array_equal(pv, wpv)


# ----------------------------------------------- method-level parity (logs)
def _logs(g, k, order, **kw):
    rp, ci = dev(g)
    c, st = kc.count(rp, ci, k, order, root_logs=True, **kw)
    lg = st["root_logs"]
    return c, st, {key: v.cpu().numpy() for key, v in lg.items()}


@pytest.mark.parametrize("order", ORDERS)
def test_root_work_logs_match_oracle(order):
    """Per-root joins and work equal the oracle's instrumented SDegree/BitCol
    (same orientation, coloring and pruning); BitCol's features too."""
    for name, g in _random_graphs(4)[:3]:
        for k in (4, 6):
            say("work logs", name, order, k)
            total, pl, per = oracle.method_count(*g, k, order)
            c, st, lg = _logs(g, k, order)
            assert c == total
            assert st["prelist_count"] == pl
            assert np.array_equal(lg["isect"], per["isect"].astype(np.int64))
            assert np.array_equal(lg["work"], per["work"].astype(np.int64))
            assert st["isect"] == int(per["isect"].sum())
            assert st["nodes"] == int(per["nodes"].sum())
            if order == "color":
                roots = per["dplus"] >= k - 1
                f = lg["features"]
                assert np.array_equal(f[roots, 0].astype(np.int64), per["dplus"][roots])
                assert np.array_equal(f[roots, 1].astype(np.int64), per["core"][roots])
                assert np.array_equal(f[roots, 2].astype(np.int64), per["colors"][roots])
                assert np.array_equal(f[roots, 3].astype(np.int64), per["edges"][roots])


@pytest.mark.parametrize("order", ["color"])
def test_schedule_does_not_change_results(order):
    """Splitting heavy roots, waves per root and queue chunking change only
    the schedule: counts, per-vertex values and per-root logs stay equal."""
    g = graphgen.chung_lu(5000, 12.0, 2.1, 600.0, planted=[40, 30, 25], seed=8)
    for k in (5, 7):
        want, wpv = oracle.count(*g, k, per_vertex=True)
        base = None
        for kw in [dict(), dict(split=1, split_threshold=1.0), dict(split=2, split_threshold=1.0),
                   dict(waves_per_root=1), dict(waves_per_root=2, chunk=3), dict(split=-1, waves_per_root=4),
                   dict(compress=-1), dict(compress=64, compress_level=2), dict(compress=20, compress_level=3),
                   dict(compress=128, compress_level=5, waves_per_root=8), dict(class_streams=1),
                   dict(class_streams=2, waves_per_root=8)]:
            say("schedule invariance", k, kw)
            c, st, lg = _logs(g, k, order, **kw)
            assert c == want, kw
            cc, pv = gpv(g, k, order, **kw)
            assert cc == want and np.array_equal(pv, wpv.astype(np.int64)), kw
            if base is None:
                base = (st, lg)
            else:
                assert np.array_equal(lg["isect"], base[1]["isect"]), kw
                assert np.array_equal(lg["work"], base[1]["work"]), kw
                assert st["nodes"] == base[0]["nodes"], kw


# Re-encoding settings (the largest set re-encoded, the lowest level, waves per
# root): off, one-word rows at every level, one-word rows from level 4 with
# the level-2 queue, and two-word rows (sets of 65..128) when counting.
REENCODE = [dict(compress=-1), dict(compress=64, compress_level=2), dict(compress=64, compress_level=4),
            dict(compress=128, compress_level=4), dict(compress=128, compress_level=3),
            dict(compress=128, compress_level=6, waves_per_root=1),
            dict(compress=100, compress_level=4, waves_per_root=4, split=2, split_threshold=1.0)]


@pytest.mark.parametrize("parts,ks", [((2,) * 64, (5, 6, 7)), ((3,) * 40, (5, 7)),
                                      ((1,) * 90 + (2,) * 10, (5, 6)), ((7, 5, 4, 3, 3, 2, 2) + (1,) * 60, (6, 8))])
def test_reencoded_nodes_closed_forms(parts, ks):
    """Dense complete multipartite graphs of 110..128 vertices: their nodes
    of level >= 4 hold up to about 125 candidates, so every re-encoding path
    runs.  Counts equal e_k of the part sizes; per-vertex values equal
    e_{k-1} of the other parts; joins and nodes do not depend on the setting."""
    (rp, ci), owner = G.multipartite(parts)
    g = (rp, ci)
    for k in ks:
        want = G.elementary_symmetric(parts, k)
        base = None
        comp = []
        for kw in REENCODE:
            say("re-encoding", len(owner), k, kw)
            c, st, lg = _logs(g, k, "color", **kw)
            assert c == want, kw
            comp.append(st["isect_compressed"])
            if base is None:
                base = (st, lg)
            else:
                assert np.array_equal(lg["isect"], base[1]["isect"]), kw
                assert np.array_equal(lg["work"], base[1]["work"]), kw
                assert st["nodes"] == base[0]["nodes"] and st["isect"] == base[0]["isect"], kw
        assert comp[0] == 0 and comp[3] >= comp[2] > 0, comp
        if k >= 6:  # children of the root's level are at level >= 4: two-word rows take them
            assert comp[3] > comp[2], comp
        say("re-encoding per-vertex", len(owner), k)
        c, pv = gpv(g, k, "color")
        assert c == want
        for i in {0, len(owner) // 2, len(owner) - 1}:
            rest = [a for j, a in enumerate(parts) if j != owner[i]]
            assert int(pv[i]) == G.elementary_symmetric(rest, k - 1)


# ------------------------------------------------------- scaled workloads
@pytest.mark.parametrize("cfg,scale,ks", [(1, 1.0, (3, 4, 5)), (2, 0.005, (5, 6)), (3, 1 / 512, (5, 6)),
                                          (5, 0.001, (5, 6))])
def test_scaled_workloads(cfg, scale, ks):
    w = graphgen.workload(cfg, scale=scale)
    g = w.graphs[0]
    for k in ks:
        want, wpv = oracle.count(*g, k, per_vertex=True)
        for order in ORDERS:
            say("workload", w.name, k, order)
            c, pv = gpv(g, k, order)
            assert c == want and np.array_equal(pv, wpv.astype(np.int64)), (w.name, k, order)


def test_batched_counts_equal_single_runs():
    """Many graphs with their own k in one call (one union graph, one listing
    launch per word class) equal the oracle graph by graph."""
    w = graphgen.workload(4, scale=0.03)
    ks = list(w.ks)
    ks[0], ks[1] = 1, 2  # the linear cases ride along
    for order in ORDERS:
        say("batched", w.name, len(w.graphs), order)
        got = kc.count_batched(w.graphs, ks, order)
        for (g, k), c in zip(zip(w.graphs, ks), got):
            assert c == oracle.count(*g, k), (k, order)


def test_plan_replays_equal_eager_and_oracle():
    """A prepared batch replayed as a captured HIP graph: every replay, with
    the program's own eager GPU work and synchronizations in between, equals
    the eager batched call and the oracle, graph by graph."""
    w = graphgen.workload(4, scale=0.03)
    ks = list(w.ks)
    ks[0], ks[1] = 1, 2
    want = [oracle.count(*g, k) for g, k in zip(w.graphs, ks)]
    assert kc.count_batched(w.graphs, ks, "color") == want
    from paper_2203_13512_amd import scheduler
    for kw in [dict(), dict(schedule="learned", mlp=scheduler.load_model(torch.device("cuda"), 8), waves_per_root=8),
               dict(compress=-1, split=2, split_threshold=1.0)]:
        say("plan", len(w.graphs), {key: v for key, v in kw.items() if key != "mlp"})
        plan = kc.plan_batched(w.graphs, ks, "color", **kw)
        try:
            for i in range(3):
                assert plan.execute() == want, (kw, i)
                x = torch.randn(1 << 20, device="cuda")
                assert float((x * 0).sum().item()) == 0.0
                torch.cuda.synchronize()
                assert kc.count_batched(w.graphs[:6], ks[:6], "color") == want[:6]
        finally:
            plan.close()
    # an overflow is reported when the plan is made
    with pytest.raises(kc.KCliqueError) as e:
        kc.plan_batched([G.complete(201)], [20], "color")
    assert e.value.status == kc.EOVERFLOW


def test_root_attribution_sums_to_the_total():
    g = graphgen.chung_lu(4000, 12.0, 2.1, 400.0, planted=[20, 12], seed=21)
    g = G.disjoint_union([g, G.complete(9), G.complete(5)])
    for order in ORDERS:
        for k in (3, 5, 7):
            say("root attribution", order, k)
            rp, ci = dev(g)
            rc = torch.zeros(len(g[0]) - 1, dtype=torch.int64, device="cuda")
            opt = kc.Options()
            kc._lib().kc_options_init(kc.ctypes.byref(opt))
            opt.device_ptrs = 1
            opt.stream = kc._torch_stream(rp.device)
            opt.root_count = rc.data_ptr()
            out = kc.ctypes.c_uint64(0)
            st = kc._lib().kclique_count_ex(len(g[0]) - 1, rp.data_ptr(), ci.data_ptr(), k, kc.ORDERS[order],
                                            kc.ctypes.byref(opt), kc.ctypes.byref(out), None)
            assert st == 0
            want = oracle.count(*g, k)
            assert out.value == want
            assert int(rc.sum().item()) == want


@pytest.mark.parametrize("order", ["degree", "core"])
def test_sdegree_split_does_not_change_results(order):
    """SDegree's heavy roots split into (root, first candidate) items: counts,
    per-vertex values, per-root joins and work and the number of calls equal
    the oracle's instrumented recursion under every split setting."""
    g = graphgen.chung_lu(5000, 12.0, 2.1, 600.0, planted=[40, 30, 25], seed=8)
    for k in (4, 6):
        want, wpv = oracle.count(*g, k, per_vertex=True)
        total, pl, per = oracle.method_count(*g, k, order)
        assert total == want
        for kw in [dict(), dict(split=-1), dict(split_threshold=1.0), dict(split_policy=1),
                   dict(split_threshold=0.5, chunk=4)]:
            say("sdegree split", order, k, kw)
            c, st, lg = _logs(g, k, order, **kw)
            assert c == want, kw
            assert np.array_equal(lg["isect"], per["isect"].astype(np.int64)), kw
            assert np.array_equal(lg["work"], per["work"].astype(np.int64)), kw
            assert st["nodes"] == int(per["nodes"].sum()), kw
            cc, pv = gpv(g, k, order, **kw)
            assert cc == want and np.array_equal(pv, wpv.astype(np.int64)), kw
