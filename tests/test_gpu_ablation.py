"""SDegree on the degeneracy order and the ablation switches (Pre-Core,
Pre-List and pruning off) against the oracle: the count never changes, and
the per-root joins and work equal the oracle's instrumented recursion run
with the same order and the same switches."""
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


GRAPHS = [
    ("chunglu", lambda: graphgen.chung_lu(5000, 10.0, 2.1, 400.0, planted=[18, 12], seed=11)),
    ("union", lambda: G.disjoint_union([G.complete(11), graphgen.erdos_renyi(120, 0.3, seed=5), G.complete(6)])),
    ("rmat", lambda: graphgen.rmat(11, 8, 0.57, 0.19, 0.19, 6, 12, 24, 0.9, seed=3)),
]


@pytest.mark.parametrize("name,make", GRAPHS, ids=[g[0] for g in GRAPHS])
@pytest.mark.parametrize("order", ["degree", "core", "color"])
def test_orders_and_ablations_match_oracle(name, make, order):
    g = make()
    rp, ci = torch.from_numpy(g[0]).cuda(), torch.from_numpy(g[1]).cuda()
    for k in (4, 6):
        want, wpv = oracle.count(*g, k, per_vertex=True)
        for disable in (0, kc.NO_PRECORE, kc.NO_PRELIST, kc.NO_PRUNE, 7):
            say(name, order, k, "disable", disable)
            total, pl, per = oracle.method_count(*g, k, order, disable=disable)
            assert total == want
            c, st = kc.count(rp, ci, k, order, root_logs=True, disable=disable)
            lg = {key: v.cpu().numpy() for key, v in st["root_logs"].items()}
            assert c == want
            assert st["prelist_count"] == pl
            assert np.array_equal(lg["isect"], per["isect"].astype(np.int64)), (order, disable)
            assert np.array_equal(lg["work"], per["work"].astype(np.int64)), (order, disable)
            assert st["nodes"] == int(per["nodes"].sum())
            c2, pv = kc.count(rp, ci, k, order, per_vertex=True, disable=disable)
            assert c2 == want and np.array_equal(pv.cpu().numpy(), wpv.astype(np.int64))


def test_unknown_ablation_bits_are_rejected():
    g = G.complete(6)
    with pytest.raises(kc.KCliqueError) as e:
        kc.count(*g, 3, "color", disable=8)
    assert e.value.status == kc.EINVAL
