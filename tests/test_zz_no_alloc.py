"""The allocation-free entry point (kclique_count_noalloc) against
kclique_count_ex, called through the C interface: same count and per-vertex
values on two calls in a row (the second on a smaller graph, so stale scratch
from the first must not matter), in both orders; a call whose scratch exceeds
the fixed array is refused with KC_EWORKSPACE."""
import ctypes
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2203_13512_amd as kc  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _call(fn, g, k, order, per_vertex):
    rp = torch.from_numpy(g[0]).cuda()
    ci = torch.from_numpy(g[1]).cuda()
    n = len(g[0]) - 1
    opt = kc.Options()
    kc._lib().kc_options_init(ctypes.byref(opt))
    opt.device_ptrs = 1
    opt.stream = kc._torch_stream(rp.device)
    out = ctypes.c_uint64(0)
    pv = torch.full((max(n, 1),), -1, dtype=torch.int64, device="cuda") if per_vertex else None
    st = fn(n, rp.data_ptr(), ci.data_ptr(), k, kc.ORDERS[order], ctypes.byref(opt), ctypes.byref(out),
            pv.data_ptr() if pv is not None else None)
    torch.cuda.synchronize()
    return st, int(out.value), (pv[:n].cpu().numpy() if pv is not None else None)


@pytest.mark.parametrize("order", ["color", "degree"])
def test_noalloc_matches_count_ex_twice_in_a_row(order):
    lib = kc._lib()
    big = graphgen.chung_lu(60000, 14.0, 2.1, 1500.0, planted=[40, 25], seed=12)
    small = graphgen.erdos_renyi(2000, 0.01, planted=[12] * 20, seed=3)
    for per_vertex in (False, True):
        for g, k in ((big, 6), (small, 4)):
            say("noalloc", order, per_vertex, len(g[0]) - 1, k)
            st0, c0, p0 = _call(lib.kclique_count_ex, g, k, order, per_vertex)
            st1, c1, p1 = _call(lib.kclique_count_noalloc, g, k, order, per_vertex)
            assert st0 == 0 and st1 == 0
            assert c1 == c0
            if per_vertex:
                assert np.array_equal(p1, p0)
    assert c0 == oracle.count(*small, 4)


def test_noalloc_refuses_calls_beyond_its_scratch():
    # 20 million vertices (one triangle among them): the per-vertex arrays of
    # the preparation alone exceed the fixed scratch
    n = 20_000_000
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = 6
    rp[1], rp[2] = 2, 4
    ci = np.array([1, 2, 0, 2, 0, 1], dtype=np.int32)
    st, c, _ = _call(kc._lib().kclique_count_noalloc, (rp, ci), 3, "color", False)
    assert st == kc.EWORKSPACE
    st, c, _ = _call(kc._lib().kclique_count_ex, (rp, ci), 3, "color", False)
    assert st == 0 and c == 1
