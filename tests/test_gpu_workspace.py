"""Caller-owned scratch: kclique_workspace_size and kc_options.workspace.

A count that takes its scratch from a torch-allocated workspace gives the same
count and per-vertex values as one where the library allocates; a workspace
one alignment unit short of the reported size is refused with KC_EWORKSPACE;
one workspace serves calls of different sizes in a row.  The MLP training step
gives bit-identical results with and without a caller workspace.
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(g):
    return torch.from_numpy(g[0]).cuda(), torch.from_numpy(g[1]).cuda()


CASES = [
    ("chunglu", lambda: graphgen.chung_lu(6000, 10.0, 2.1, 500.0, planted=[22, 16], seed=3), (4, 6)),
    ("minus_edge", lambda: G.complete_minus_edge(90, 5, 9), (5,)),
    ("union", lambda: G.disjoint_union([G.complete(12), graphgen.erdos_renyi(90, 0.35, seed=2)]), (3, 5)),
]


@pytest.mark.parametrize("order", ["color", "degree"])
@pytest.mark.parametrize("name,make,ks", CASES, ids=[c[0] for c in CASES])
def test_workspace_gives_identical_results(order, name, make, ks):
    g = make()
    rp, ci = dev(g)
    for k in ks:
        for per_vertex in (False, True):
            say("workspace", name, order, k, per_vertex)
            want = oracle.count(*g, k, per_vertex=per_vertex)
            nbytes = kc.workspace_size(rp, ci, k, order, per_vertex=per_vertex)
            assert nbytes > 0 and nbytes % 256 == 0
            ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            got = kc.count(rp, ci, k, order, per_vertex=per_vertex, workspace=ws)
            if per_vertex:
                assert got[0] == want[0]
                assert np.array_equal(got[1].cpu().numpy(), want[1].astype(np.int64))
            else:
                assert got == want
            # host arrays: the CSR copies come from the workspace too
            nb_host = kc.workspace_size(*g, k, order, per_vertex=per_vertex)
            assert nb_host >= nbytes
            wsh = torch.empty(nb_host, dtype=torch.uint8, device="cuda")
            goth = kc.count(*g, k, order, per_vertex=per_vertex, workspace=wsh)
            assert (goth[0] if per_vertex else goth) == (want[0] if per_vertex else want)
            small = ws[: nbytes - 256]
            with pytest.raises(kc.KCliqueError) as e:
                kc.count(rp, ci, k, order, per_vertex=per_vertex, workspace=small)
            assert e.value.status == kc.EWORKSPACE


def test_workspace_reused_across_calls_and_schedules():
    from paper_2203_13512_amd import scheduler
    big = graphgen.chung_lu(20000, 12.0, 2.1, 800.0, planted=[30, 24], seed=5)
    small = graphgen.erdos_renyi(400, 0.06, planted=[14, 11], seed=1)
    mlp = scheduler.load_model(torch.device("cuda"), 6)
    kw = dict(schedule="learned", mlp=mlp, split=2, split_threshold=1.0)
    need = max(kc.workspace_size(*dev(big), 6, "color", **kw), kc.workspace_size(*dev(small), 6, "color", **kw))
    ws = torch.full((need,), 0xA5, dtype=torch.uint8, device="cuda")  # stale contents must not matter
    for g in (big, small, big):
        say("reuse", len(g[0]) - 1)
        want = oracle.count(*g, 6)
        assert kc.count(*dev(g), 6, "color", workspace=ws, **kw) == want
        assert kc.count(*dev(g), 6, "color", workspace="torch") == want


def test_mlp_training_step_with_workspace_is_bit_identical():
    rng = np.random.default_rng(0)
    rows = 1000
    X = torch.tensor(rng.normal(size=(rows, 4)).astype(np.float32), device="cuda")
    T = torch.tensor(rng.normal(size=rows).astype(np.float32), device="cuda")
    from paper_2203_13512_amd import scheduler
    P0 = torch.tensor(scheduler.init_params(1), device="cuda")
    nbytes = kc.mlp_workspace_size(rows)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    runs = []
    for w in (None, ws):
        P = P0.clone()
        m = torch.zeros_like(P)
        v = torch.zeros_like(P)
        for t in range(1, 4):
            loss, grad = kc.mlp_train_step(P, X, T, m, v, t=t, lr=1e-2, workspace=w)
        torch.cuda.synchronize()
        runs.append((P.cpu().numpy(), grad.cpu().numpy(), loss.cpu().numpy()))
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)
    with pytest.raises(kc.KCliqueError) as e:
        kc.mlp_train_step(P0.clone(), X, T, workspace=ws[: nbytes - 256])
    assert e.value.status == kc.EWORKSPACE
