"""Root shares (kc_options.root_mask): the listing restricted to a set of
roots.  Theorem 1 gives every k-clique exactly one root (its first vertex in
the orientation), so the share of the roots in a mask lists exactly the
cliques rooted there, and the Pre-List cliques of a clique component (Alg. 4)
belong to the share of its smallest vertex.

Each share's count equals the oracle's per-root counts summed over the
share (plus its Pre-List components); the shares of a partition add up to the
oracle's total, per-vertex participation and listing, in every order.
"""
import sys

import numpy as np
import pytest

import graphgen
import oracle
from tests import _graphs as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2203_13512_amd as kc  # noqa: E402
from paper_2203_13512_amd import scheduler  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(g):
    rp, ci = g
    return (torch.from_numpy(np.ascontiguousarray(rp, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(ci, dtype=np.int32)).cuda())


def shares_of(n, S, seed=0):
    """Share index of every vertex: a multiplicative hash of its id, so that
    heavy and light roots spread over the shares."""
    u = np.arange(n, dtype=np.uint64) + np.uint64(seed)
    return (((u * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)) * np.uint64(S) >> np.uint64(32)).astype(np.int64)


def prelist_components(rp, ci, k):
    """(smallest vertex, size) of every clique component Pre-List removes,
    from the oracle's Pre-Core and Pre-List: the vertices Pre-List removes,
    grouped by connectivity (each group is a whole component of the graph)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    rem0 = oracle.precore(rp, ci, k).astype(bool)
    rem1, pl, _, _ = oracle.prelist(rp, ci, k, rem0.astype(np.uint8))
    gone = rem1.astype(bool) & ~rem0
    n = len(rp) - 1
    src = np.repeat(np.arange(n), np.diff(rp))
    keep = gone[src] & gone[ci]
    A = csr_matrix((np.ones(int(keep.sum())), (src[keep], ci[keep])), shape=(n, n))
    _, lab = connected_components(A, directed=False)
    comps = []
    for c in np.unique(lab[gone]):
        mem = np.flatnonzero(gone & (lab == c))
        comps.append((int(mem.min()), len(mem)))
    assert sum(oracle.binom(s, k) for _, s in comps) == pl
    return comps


def expected_share_counts(g, k, order, share, S):
    total, _, per = oracle.method_count(*g, k, order)
    roots = per["dplus"] >= k - 1
    want = np.zeros(S, dtype=object)
    for s in range(S):
        want[s] = int(per["count"][roots & (share == s)].astype(np.uint64).sum())
    for v, size in prelist_components(*g, k):
        want[share[v]] += oracle.binom(size, k)
    assert sum(want) == total
    return [int(x) for x in want], total


GRAPHS = [
    ("er", lambda: graphgen.erdos_renyi(400, 0.06, planted=[14, 11, 9], seed=3)),
    ("chunglu", lambda: graphgen.chung_lu(6000, 10.0, 2.1, 500.0, planted=[22, 16], seed=3)),
    ("rmat", lambda: graphgen.rmat(11, 8, 0.57, 0.19, 0.19, 6, 12, 24, 0.9, seed=3)),
    # two clique components (Pre-List) beside a dense random part
    ("union", lambda: G.disjoint_union([G.complete(12), graphgen.erdos_renyi(90, 0.35, seed=3), G.complete(6),
                                        G.complete(9)])),
    ("bipartite", lambda: G.bipartite_with_clique(200, 150, 9)),
]
ORDERS = ["degree", "color", "core", "degree_reduced"]


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("name,make", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_share_counts_match_oracle(order, name, make):
    g = make()
    rp, ci = dev(g)
    n = len(g[0]) - 1
    S = 3
    share = shares_of(n, S)
    share_d = torch.from_numpy(share).cuda()
    for k in (3, 4, 6):
        want, total = expected_share_counts(g, k, order, share, S)
        _, wpv = oracle.count(*g, k, per_vertex=True)
        for kw in (dict(), dict(split=1, split_threshold=1.0)):
            say("shares", name, order, k, kw, want)
            pv_sum = torch.zeros(n, dtype=torch.int64, device="cuda")
            for s in range(S):
                m = share_d == s
                c = kc.count(rp, ci, k, order, root_mask=m, **kw)
                assert c == want[s], (s, kw)
                c2, pv = kc.count(rp, ci, k, order, per_vertex=True, root_mask=m, **kw)
                assert c2 == want[s]
                assert int(pv.sum()) == k * c2
                pv_sum += pv
            assert np.array_equal(pv_sum.cpu().numpy(), wpv.astype(np.int64)), kw
        # every vertex in the mask: the unmasked call; no vertex: nothing
        assert kc.count(rp, ci, k, order, root_mask=torch.ones(n, dtype=torch.bool, device="cuda")) == total
        assert kc.count(rp, ci, k, order, root_mask=torch.zeros(n, dtype=torch.bool, device="cuda")) == 0


@pytest.mark.parametrize("order", ["degree", "color"])
def test_share_listings_partition_the_oracle_listing(order):
    for name, make in GRAPHS:
        g = make()
        rp, ci = dev(g)
        n = len(g[0]) - 1
        share = torch.from_numpy(shares_of(n, 4, seed=5)).cuda()
        for k in (3, 5):
            if oracle.count(*g, k) > 200000:
                continue
            exp, total = oracle.list_cliques(*g, k)
            say("share listing", name, order, k, total)
            rows = []
            for s in range(4):
                r, t = kc.list_cliques(rp, ci, k, order, root_mask=share == s)
                assert len(r) == t
                rows.append(r.cpu().numpy())
            got = np.sort(np.concatenate(rows), axis=1)
            assert len(got) == total
            assert np.array_equal(got[np.lexsort(got.T[::-1])], np.asarray(exp, dtype=np.int32))


def test_learned_schedule_and_wide_roots_in_shares():
    """K_n minus one edge keeps its roots (Pre-List does not apply); at n = 700
    the roots fill the 1- to 24-word classes.  Shares under the learned
    schedule add up to C(n, k) - C(n-2, k-2)."""
    n = 700
    g = G.complete_minus_edge(n, 3, 650)
    rp, ci = dev(g)
    mlp = scheduler.load_model(torch.device("cuda"), 5)
    want = oracle.binom(n, 5) - oracle.binom(n - 2, 3)
    share = torch.from_numpy(shares_of(n, 5)).cuda()
    for kw in (dict(schedule="learned", mlp=mlp), dict(schedule="degree")):
        parts = [kc.count(rp, ci, 5, "color", root_mask=share == s, **kw) for s in range(5)]
        say("wide shares", {key: v for key, v in kw.items() if key != "mlp"}, parts)
        assert sum(parts) == want and all(p > 0 for p in parts)


def test_root_mask_refusals():
    import ctypes
    g = G.complete(8)
    rp, ci = dev(g)
    m = torch.ones(8, dtype=torch.uint8, device="cuda")
    with pytest.raises(kc.KCliqueError) as e:
        kc.count(rp, ci, 2, "color", root_mask=m)
    assert e.value.status == kc.EUNSUPPORTED
    with pytest.raises(ValueError):
        kc.count(rp, ci, 4, "color", root_mask=torch.ones(7, dtype=torch.uint8, device="cuda"))
    # through the C-ABI: a mask with host graph arrays, and with a batch
    L = kc._lib()
    opt = kc.Options()
    L.kc_options_init(ctypes.byref(opt))
    opt.root_mask = m.data_ptr()
    rp_h = np.ascontiguousarray(g[0], dtype=np.int32)
    ci_h = np.ascontiguousarray(g[1], dtype=np.int32)
    out = ctypes.c_uint64(0)
    assert L.kclique_count_ex(8, rp_h.ctypes.data, ci_h.ctypes.data, 4, kc.ORDERS["color"], ctypes.byref(opt),
                              ctypes.byref(out), None) == kc.EINVAL
    nn = np.array([8], dtype=np.int32)
    ro = np.array([0], dtype=np.int64)
    co = np.array([0], dtype=np.int64)
    kk = np.array([4], dtype=np.int32)
    counts = np.zeros(1, dtype=np.uint64)
    assert L.kclique_count_batched(1, nn.ctypes.data, ro.ctypes.data, co.ctypes.data, rp_h.ctypes.data,
                                   ci_h.ctypes.data, kk.ctypes.data, kc.ORDERS["color"], ctypes.byref(opt),
                                   counts.ctypes.data) == kc.EINVAL


def test_full_size_workload_2_in_shares():
    """Workload 2 (Chung-Lu, 1M vertices) at k = 5 in 4 root shares: the
    shares add up to the oracle's golden count, in both methods."""
    import json
    import os
    with open(os.path.join(G.GOLDEN, "fullsize_w2_k5_degree.json")) as f:
        gold = json.load(f)
    w = G.workload_cached(2)
    rp_h, ci_h = w.graphs[0]
    assert G.graph_sha(rp_h, ci_h) == gold["graph_sha256"]
    rp, ci = dev((rp_h, ci_h))
    share = torch.from_numpy(shares_of(len(rp_h) - 1, 4)).cuda()
    mlp = scheduler.load_model(rp.device, 5)
    for order, kw in (("color", dict(schedule="learned", mlp=mlp)), ("degree_reduced", dict())):
        parts = [kc.count(rp, ci, 5, order, root_mask=share == s, **kw) for s in range(4)]
        say("workload 2, k = 5, shares", order, parts)
        assert sum(parts) == gold["count"]
