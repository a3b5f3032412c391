"""Wide local subgraphs: every bitmap word class of the BitCol listing kernel
(1 to 64 words of 32 bits, local subgraphs of up to 2048 vertices; the widest
classes keep their bitmaps in device memory) and every candidate-list class of
SDegree, including its device-memory lists, against closed forms.

K_n minus one edge survives Pre-Core and Pre-List (it is not a clique), and
under the degeneracy order its roots have every out-degree from 0 to n-2, so
one graph puts roots into every word class; its k-cliques number
C(n,k) - C(n-2,k-2).  The cocktail-party graph K_{2 x r} (every vertex
adjacent to all but its partner) has 2^k C(r,k) of them and 2^(k-1) C(r-1,k-1)
per vertex.  The statistics' per-class task counts show which word classes
ran.
"""
import math
import sys

import numpy as np
import pytest

from tests import _graphs as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2203_13512_amd as kc  # noqa: E402

WORDS = [1, 2, 4, 8, 12, 16, 24, 32, 48, 64]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(g):
    rp, ci = g
    return torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()


def minus_edge_count(n, k):
    return math.comb(n, k) - math.comb(n - 2, k - 2)


def minus_edge_pv(n, k, a=0, b=1):
    pv = np.full(n, math.comb(n - 1, k - 1) - math.comb(n - 3, k - 3), dtype=np.int64)
    pv[[a, b]] = math.comb(n - 2, k - 1)
    return pv


def classes_run(st):
    return [WORDS[c] for c in range(10) if st["class_tasks"][c] > 0]


LAUNCH = [dict(), dict(waves_per_root=1), dict(waves_per_root=4, chunk=4), dict(compress=-1),
          dict(compress=64, compress_level=3), dict(split=1, split_threshold=1.0),
          dict(split=2, split_threshold=1.0, waves_per_root=8), dict(class_streams=2),
          dict(waves_per_root=16), dict(waves_per_root=16, split=2, split_threshold=1.0)]


@pytest.mark.parametrize("k", [4, 5])
def test_every_word_class_complete_minus_edge(k):
    n = 1000
    g = dev(G.complete_minus_edge(n))
    want = minus_edge_count(n, k)
    # every launch shape at k = 4; at k = 5 (40x the joins) three of them
    base = None
    for kw in (LAUNCH if k == 4 else [dict(), dict(split=2, split_threshold=1.0, waves_per_root=8),
                                      dict(class_streams=2), dict(waves_per_root=16)]):
        say("K_n - e", n, k, kw)
        c, st = kc.count(*g, k, "color", stats=True, **kw)
        assert c == want, kw
        assert classes_run(st) == WORDS[:8], classes_run(st)
        assert st["max_out_degree"] == n - 2
        # joins and nodes are the method's, whatever the launch shape
        base = base or st
        assert (st["isect"], st["nodes"]) == (base["isect"], base["nodes"]), kw


def test_every_word_class_k6_and_learned_schedule():
    from paper_2203_13512_amd import scheduler
    n = 400
    g = dev(G.complete_minus_edge(n, 7, 300))
    mlp = scheduler.load_model(torch.device("cuda"), 6)
    for kw in [dict(), dict(schedule="learned", mlp=mlp), dict(compress=-1, waves_per_root=8)]:
        say("K_n - e", n, 6, {key: v for key, v in kw.items() if key != "mlp"})
        c, st = kc.count(*g, 6, "color", stats=True, **kw)
        assert c == minus_edge_count(n, 6)
        assert classes_run(st) == [1, 2, 4, 8, 12, 16]


@pytest.mark.parametrize("k", [4, 5])
def test_every_word_class_cocktail_party(k):
    r = 500
    g = dev(G.cocktail_party(r))
    for kw in ([dict(), dict(compress=-1), dict(waves_per_root=4, split=2, split_threshold=1.0)] if k == 4
               else [dict(waves_per_root=4, split=2, split_threshold=1.0)]):
        say("cocktail party", r, k, kw)
        c, st = kc.count(*g, k, "color", stats=True, **kw)
        assert c == 2 ** k * math.comb(r, k), kw
        assert classes_run(st) == WORDS[:8]


@pytest.mark.parametrize("k", [4, 5])
def test_per_vertex_up_to_512_local_vertices(k):
    n = 514  # out-degrees up to 512: every per-vertex word class (1..16 words)
    g = dev(G.complete_minus_edge(n, 3, 400))
    for kw in [dict(), dict(compress=-1), dict(waves_per_root=8, split=1, split_threshold=1.0)]:
        say("per-vertex K_n - e", n, k, kw)
        c, pv, st = kc.count(*g, k, "color", per_vertex=True, stats=True, **kw)
        assert c == minus_edge_count(n, k)
        assert np.array_equal(pv.cpu().numpy(), minus_edge_pv(n, k, 3, 400)), kw
        assert classes_run(st) == [1, 2, 4, 8, 12, 16]
    r = 257
    c, pv = kc.count(*dev(G.cocktail_party(r)), k, "color", per_vertex=True)
    assert c == 2 ** k * math.comb(r, k)
    assert bool((pv == 2 ** (k - 1) * math.comb(r - 1, k - 1)).all())


def test_sdegree_list_classes_above_1024():
    """Degree order: out-degrees above 1024 take SDegree's 4096-entry
    candidate-list class (lists sized by the class's largest out-degree,
    here in LDS)."""
    n = 1030
    g = dev(G.complete_minus_edge(n))
    c, st = kc.count(*g, 4, "degree", stats=True)
    assert c == minus_edge_count(n, 4)
    assert st["max_out_degree"] == n - 2 and st["class_tasks"][3] > 0
    c, pv = kc.count(*g, 4, "degree", per_vertex=True)
    assert c == minus_edge_count(n, 4)
    assert np.array_equal(pv.cpu().numpy(), minus_edge_pv(n, 4))


@pytest.mark.skip(reason="faulted the GPU once (a KCliqueError after a device fault; the sub-case was not "
                         "identified).  The paths it exercised for the first time -- BitCol's device-memory "
                         "classes above k = 5 and SDegree's device-memory lists with per-vertex or listing "
                         "output -- are refused by the library (KC_EUNSUPPORTED) until the cause is found")
def test_sdegree_device_memory_lists():
    """Degree order, k = 16 and out-degrees of 1030: a workgroup's 16 levels
    of 1088-entry lists exceed 64 KiB of LDS and live in device memory.
    K_{1030,1030} plus a 15-clique on the right: every left vertex roots one
    16-clique (itself and the clique)."""
    a = b = 1030
    m = 15
    k = 16
    g_h = G.bipartite_with_clique(a, b, m)
    g = dev(g_h)
    want = a * math.comb(m, k - 1) + math.comb(m, k)
    pv_want = np.zeros(a + b, dtype=np.int64)
    pv_want[:a] = math.comb(m, k - 1)
    pv_want[a:a + m] = a * math.comb(m - 1, k - 2) + math.comb(m - 1, k - 1)
    for order in ("degree", "core", "color"):
        for kw in (dict(), dict(disable=kc.NO_PRUNE), dict(split=1, split_threshold=1.0)):
            say("bipartite + clique", order, kw)
            c, st = kc.count(*g, k, order, stats=True, **kw)
            assert c == want, (order, kw)
            if order == "degree":
                assert st["max_out_degree"] == b and st["class_tasks"][3] >= a  # roots or edge tasks
        c, pv = kc.count(*g, k, order, per_vertex=True)
        assert c == want and np.array_equal(pv.cpu().numpy(), pv_want), order
        rows, total = kc.list_cliques(*g, k, order)
        assert total == want
        r = np.sort(rows.cpu().numpy(), axis=1)
        assert sorted(map(tuple, r)) == [tuple([u] + list(range(a, a + m))) for u in range(a)]


def test_unvalidated_device_memory_paths_are_refused():
    """The device-memory bitmap classes (above 1024 local vertices, above 512
    with per-vertex output) run up to k = 5 only, and SDegree's device-memory
    lists only when counting; beyond that the call returns KC_EUNSUPPORTED
    before any listing kernel runs."""
    n = 1030
    g = dev(G.complete_minus_edge(n))
    for k, pv in ((6, False), (7, False)):
        with pytest.raises(kc.KCliqueError) as e:
            kc.count(*g, k, "color", per_vertex=pv)
        assert e.value.status == kc.EUNSUPPORTED
    g8 = dev(G.complete_minus_edge(600, 0, 500))
    with pytest.raises(kc.KCliqueError) as e:
        kc.count(*g8, 6, "color", per_vertex=True)
    assert e.value.status == kc.EUNSUPPORTED
    # k = 16: 16 levels of 1088-entry lists do not fit LDS
    with pytest.raises(kc.KCliqueError) as e:
        kc.count(*g, 16, "degree", per_vertex=True)
    assert e.value.status == kc.EUNSUPPORTED
    with pytest.raises(kc.KCliqueError) as e:
        kc.list_cliques(*g, 16, "degree", capacity=10)
    assert e.value.status == kc.EUNSUPPORTED


@pytest.mark.parametrize("n", [1030, 1600, 2050])
def test_local_subgraphs_in_device_memory(n):
    """Local subgraphs of 1025..2048 vertices (48- and 64-word bitmaps) are
    staged and listed with their bitmaps in device memory; per-vertex output
    above 512 local vertices (24 and 32 words and beyond) likewise."""
    g = dev(G.complete_minus_edge(n, 2, n - 3))
    for kw in [dict(), dict(waves_per_root=1), dict(compress=-1), dict(split=2, split_threshold=1.0)]:
        say("device-memory bitmaps", n, kw)
        c, st = kc.count(*g, 4, "color", stats=True, **kw)
        assert c == minus_edge_count(n, 4), kw
        assert st["max_out_degree"] == n - 2
        assert st["class_tasks"][8 if n <= 1538 else 9] > 0
    c, pv = kc.count(*g, 4, "color", per_vertex=True)
    assert c == minus_edge_count(n, 4)
    assert np.array_equal(pv.cpu().numpy(), minus_edge_pv(n, 4, 2, n - 3))
    # listing from the device-memory classes: a bounded buffer of valid,
    # distinct triangles (the missing edge (2, n-3) is in none of them)
    rows, total = kc.list_cliques(*g, 3, "color", capacity=1000)
    assert total == minus_edge_count(n, 3) and rows.shape == (1000, 3)
    r = np.sort(rows.cpu().numpy(), axis=1)
    assert len({tuple(x) for x in r}) == 1000
    assert np.all((r[:, 0] < r[:, 1]) & (r[:, 1] < r[:, 2]) & (r[:, 0] >= 0) & (r[:, 2] < n))
    assert not np.any(np.isin(r, [2]).any(axis=1) & np.isin(r, [n - 3]).any(axis=1))


def test_per_vertex_classes_beyond_512_local_vertices():
    n = 800  # out-degrees up to 798: per-vertex classes of 24 and 32 words
    g = dev(G.complete_minus_edge(n, 0, 500))
    for k in (4, 5):
        c, pv, st = kc.count(*g, k, "color", per_vertex=True, stats=True)
        assert c == minus_edge_count(n, k)
        assert np.array_equal(pv.cpu().numpy(), minus_edge_pv(n, k, 0, 500))
        assert st["class_tasks"][6] > 0 and st["class_tasks"][7] > 0


def test_local_subgraphs_beyond_the_supported_size_are_reported():
    """Local subgraphs of more than 2048 vertices are refused, not truncated."""
    g = dev(G.complete_minus_edge(2060))
    with pytest.raises(kc.KCliqueError) as e:
        kc.count(*g, 3, "color")
    assert e.value.status == kc.EUNSUPPORTED
