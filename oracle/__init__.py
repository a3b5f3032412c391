"""CPU oracle for exact k-clique counting -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The GPU library never calls it, and it shares no
code with the GPU library: the C source ``kc_oracle.c`` is written directly
from the paper's definitions and algorithms (see its header for the passage
each function follows and the readings taken where the paper is ambiguous).

Parity status: every function here is pinned by tests in
``tests/test_oracle_pins.py`` (closed forms, brute force, the paper's worked
examples).  The per-root work counters have no values printed in the paper;
they are pinned by hand-derived traces of the paper's own examples (SDegree's
recursion of Example 4, BitCol's Alg. 6 on the Example 6 / Table 3 local
graph) and by the Lemma 4 bound.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kc_oracle.c")
_LIB = os.path.join(_HERE, "libkcoracle.so")
_lib = None

OK, EINVAL, ENOMEM, EOVERFLOW, EBUDGET = 0, -1, -2, -3, -6


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    L = ctypes.CDLL(_LIB)
    i32, u64, i64, dbl, vp = ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    sig = {
        "orc_binom": [u64, u64, vp],
        "orc_validate": [i32, vp, vp],
        "orc_count_brute": [i32, vp, vp, i32, vp, vp],
        "orc_count_idorder": [i32, vp, vp, i32, vp, vp],
        "orc_count_idorder_roots": [i32, vp, vp, i32, vp, i32, dbl, vp, vp, vp],
        "orc_vertex_count": [i32, vp, vp, i32, i32, u64, vp],
        "orc_list_idorder": [i32, vp, vp, i32, vp, i64, vp, vp],
        "orc_core_numbers": [i32, vp, vp, vp],
        "orc_precore": [i32, vp, vp, i32, vp],
        "orc_prelist": [i32, vp, vp, i32, vp, vp, vp, vp],
        "orc_degree_dag": [i32, vp, vp, vp, vp, vp],
        "orc_degeneracy_dag": [i32, vp, vp, vp, vp, vp, vp, vp],
        "orc_sdegree_dag": [i32, vp, vp, i32, vp, vp, vp, vp, vp],
        "orc_sdegree_reduced_dag": [i32, vp, vp, i32, vp, vp, vp, vp, vp],
        "orc_greedy_color": [i32, vp, vp, vp, vp],
        "orc_bitcol_encode": [i32, vp, vp, i32, vp, vp],
        "orc_bitcol_dag": [i32, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp],
        "orc_bitcol_roots": [i32, vp, vp, i32, i32, i32, vp, vp, vp, vp, vp],
        "orc_bitcol_roots_timed": [i32, vp, vp, i32, i32, i32, vp, dbl, vp, vp],
        "orc_sdegree_roots_timed": [i32, vp, vp, i32, i32, i32, vp, dbl, vp, vp],
        "orc_sdegree_roots": [i32, vp, vp, i32, i32, vp, vp, vp, vp, vp],
        "orc_sdegree_reduced_roots": [i32, vp, vp, i32, i32, vp, vp, vp, vp, vp],
        "orc_merge_join": [vp, i32, vp, i32, vp],
        "orc_method_count": [i32, vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    _lib = L
    return L


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _csr(rp, ci):
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, dtype=np.int32)
    return rp, ci


def _check(st, what):
    if st != OK:
        raise OracleError(st, what)


def binom(n: int, k: int):
    """C(n, k) as a Python int, or None when it does not fit in uint64."""
    out = np.zeros(1, dtype=np.uint64)
    st = _load().orc_binom(n, k, _p(out))
    if st == EOVERFLOW:
        return None
    _check(st, "binom")
    return int(out[0])


def validate(rp, ci) -> bool:
    rp, ci = _csr(rp, ci)
    return _load().orc_validate(len(rp) - 1, _p(rp), _p(ci)) == OK


def count_brute(rp, ci, k: int, per_vertex: bool = False):
    rp, ci = _csr(rp, ci)
    n = len(rp) - 1
    c = np.zeros(1, dtype=np.uint64)
    pv = np.zeros(max(n, 1), dtype=np.uint64) if per_vertex else None
    _check(_load().orc_count_brute(n, _p(rp), _p(ci), k, _p(c), _p(pv)), "count_brute")
    return (int(c[0]), pv[:n]) if per_vertex else int(c[0])


def count(rp, ci, k: int, per_vertex: bool = False):
    """Exact k-clique count (and per-vertex participation) by the ordered
    recursion over vertex ids."""
    rp, ci = _csr(rp, ci)
    n = len(rp) - 1
    c = np.zeros(1, dtype=np.uint64)
    pv = np.zeros(max(n, 1), dtype=np.uint64) if per_vertex else None
    _check(_load().orc_count_idorder(n, _p(rp), _p(ci), k, _p(c), _p(pv)), "count")
    return (int(c[0]), pv[:n]) if per_vertex else int(c[0])


def count_roots(rp, ci, k: int, roots, seconds: float = 0.0):
    """Cliques whose smallest vertex id is in `roots`, optionally stopping at a
    time limit.  Returns (count, roots_completed, finished)."""
    rp, ci = _csr(rp, ci)
    n = len(rp) - 1
    r = np.ascontiguousarray(roots, dtype=np.int32)
    c = np.zeros(1, dtype=np.uint64)
    done = np.zeros(1, dtype=np.int32)
    st = _load().orc_count_idorder_roots(n, _p(rp), _p(ci), k, _p(r), len(r), float(seconds), _p(c), None, _p(done))
    if st not in (OK, EBUDGET):
        _check(st, "count_roots")
    return int(c[0]), int(done[0]), st == OK


def list_cliques(rp, ci, k: int, capacity: int | None = None):
    """Every k-clique as a row of ascending vertex ids (rows in the order of
    the ordered recursion, i.e. lexicographic).  Returns (rows, total)."""
    rp, ci = _csr(rp, ci)
    n = len(rp) - 1
    if capacity is None:
        capacity = count(rp, ci, k)
    out = np.zeros(max(capacity * k, 1), dtype=np.int32)
    written = np.zeros(1, dtype=np.int64)
    total = np.zeros(1, dtype=np.uint64)
    _check(_load().orc_list_idorder(n, _p(rp), _p(ci), k, _p(out), capacity, _p(written), _p(total)), "list_cliques")
    return out[: int(written[0]) * k].reshape(-1, k), int(total[0])


def vertex_count(rp, ci, k: int, v: int, budget: int = 0):
    """Number of k-cliques containing v, or None if over the budget."""
    rp, ci = _csr(rp, ci)
    out = np.zeros(1, dtype=np.uint64)
    st = _load().orc_vertex_count(len(rp) - 1, _p(rp), _p(ci), k, v, budget, _p(out))
    if st == EBUDGET:
        return None
    _check(st, "vertex_count")
    return int(out[0])


def core_numbers(rp, ci) -> np.ndarray:
    rp, ci = _csr(rp, ci)
    n = len(rp) - 1
    core = np.zeros(max(n, 1), dtype=np.int32)
    _check(_load().orc_core_numbers(n, _p(rp), _p(ci), _p(core)), "core_numbers")
    return core[:n]


def precore(rp, ci, k: int) -> np.ndarray:
    rp, ci = _csr(rp, ci)
    n = len(rp) - 1
    removed = np.zeros(max(n, 1), dtype=np.uint8)
    _check(_load().orc_precore(n, _p(rp), _p(ci), k, _p(removed)), "precore")
    return removed[:n]


def prelist(rp, ci, k: int, removed: np.ndarray, per_vertex: bool = False):
    """Returns (removed_after, count, per_vertex or None, clique_components)."""
    rp, ci = _csr(rp, ci)
    n = len(rp) - 1
    rem = np.ascontiguousarray(removed, dtype=np.uint8).copy()
    if rem.size == 0:
        rem = np.zeros(1, dtype=np.uint8)
    c = np.zeros(1, dtype=np.uint64)
    pv = np.zeros(max(n, 1), dtype=np.uint64) if per_vertex else None
    nc = np.zeros(1, dtype=np.int32)
    _check(_load().orc_prelist(n, _p(rp), _p(ci), k, _p(rem), _p(c), _p(pv), _p(nc)), "prelist")
    return rem[:n], int(c[0]), (pv[:n] if per_vertex else None), int(nc[0])


def degree_dag(rp, ci, removed):
    rp, ci = _csr(rp, ci)
    n = len(rp) - 1
    rem = np.ascontiguousarray(removed, dtype=np.uint8)
    drp = np.zeros(n + 1, dtype=np.int32)
    dci = np.zeros(len(ci) // 2 + 1, dtype=np.int32)
    _check(_load().orc_degree_dag(n, _p(rp), _p(ci), _p(rem), _p(drp), _p(dci)), "degree_dag")
    return drp, dci[: drp[-1]]


def degeneracy_dag(rp, ci, removed):
    """Returns (dag_rp, dag_col, round, core) of the synchronous peel."""
    rp, ci = _csr(rp, ci)
    n = len(rp) - 1
    rem = np.ascontiguousarray(removed, dtype=np.uint8)
    drp = np.zeros(n + 1, dtype=np.int32)
    dci = np.zeros(len(ci) // 2 + 1, dtype=np.int32)
    rnd = np.zeros(max(n, 1), dtype=np.int32)
    core = np.zeros(max(n, 1), dtype=np.int32)
    _check(_load().orc_degeneracy_dag(n, _p(rp), _p(ci), _p(rem), _p(drp), _p(dci), _p(rnd), _p(core)),
           "degeneracy_dag")
    return drp, dci[: drp[-1]], rnd[:n], core[:n]


def merge_join(a, b) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.int32)
    b = np.ascontiguousarray(b, dtype=np.int32)
    out = np.zeros(max(len(a), len(b), 1), dtype=np.int32)
    m = _load().orc_merge_join(_p(a), len(a), _p(b), len(b), _p(out))
    return out[:m]


def sdegree_dag(drp, dci, k: int, reduce: bool = False):
    """SDegree (Alg. 5) from every root of the DAG; with `reduce`, on each
    root's induced DAG G_u (the out-neighbour reduction of Sec. 7.2)."""
    drp, dci = _csr(drp, dci)
    n = len(drp) - 1
    c = np.zeros(1, dtype=np.uint64)
    arrs = [np.zeros(max(n, 1), dtype=np.uint64) for _ in range(4)]
    fn = _load().orc_sdegree_reduced_dag if reduce else _load().orc_sdegree_dag
    _check(fn(n, _p(drp), _p(dci), k, _p(c), *[_p(a) for a in arrs]), "sdegree_dag")
    return int(c[0]), dict(zip(["count", "nodes", "isect", "elems"], [a[:n] for a in arrs]))


def sdegree_roots(drp, dci, k: int, roots, reduce: bool = False):
    """SDegree from the listed roots of the DAG only; dict of per-root arrays
    (count, nodes, isect, elems) in the order of `roots`."""
    drp, dci = _csr(drp, dci)
    n = len(drp) - 1
    roots = np.ascontiguousarray(roots, dtype=np.int32)
    r = max(len(roots), 1)
    u = [np.zeros(r, dtype=np.uint64) for _ in range(4)]
    fn = _load().orc_sdegree_reduced_roots if reduce else _load().orc_sdegree_roots
    _check(fn(n, _p(drp), _p(dci), k, len(roots), _p(roots), *[_p(a) for a in u]), "sdegree_roots")
    return dict(zip(["count", "nodes", "isect", "elems"], [a[:len(roots)] for a in u]))


def greedy_color(adj: np.ndarray, ids):
    adj = np.ascontiguousarray(adj, dtype=np.uint8)
    s = adj.shape[0]
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    order = np.zeros(max(s, 1), dtype=np.int32)
    color = np.zeros(max(s, 1), dtype=np.int32)
    _check(_load().orc_greedy_color(s, _p(adj), _p(ids), _p(order), _p(color)), "greedy_color")
    return order[:s], color[:s]


def bitcol_encode(adj: np.ndarray, ids, L: int):
    adj = np.ascontiguousarray(adj, dtype=np.uint8)
    s = adj.shape[0]
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    nw = (s + L - 1) // L
    color = np.zeros(max(s, 1), dtype=np.int32)
    B = np.zeros(max(s * nw, 1), dtype=np.uint32)
    _check(_load().orc_bitcol_encode(s, _p(adj), _p(ids), L, _p(color), _p(B)), "bitcol_encode")
    return color[:s], B[: s * nw].reshape(s, nw)


def bitcol_dag(drp, dci, k: int, L: int = 32):
    drp, dci = _csr(drp, dci)
    n = len(drp) - 1
    c = np.zeros(1, dtype=np.uint64)
    u = [np.zeros(max(n, 1), dtype=np.uint64) for _ in range(4)]
    colors = np.zeros(max(n, 1), dtype=np.int32)
    edges = np.zeros(max(n, 1), dtype=np.int64)
    _check(_load().orc_bitcol_dag(n, _p(drp), _p(dci), k, L, _p(c), *[_p(a) for a in u], _p(colors), _p(edges)),
           "bitcol_dag")
    d = dict(zip(["count", "nodes", "isect", "words"], [a[:n] for a in u]))
    d["colors"] = colors[:n]
    d["edges"] = edges[:n]
    return int(c[0]), d


def bitcol_count_roots(drp, dci, k: int, roots, seconds: float, L: int = 32):
    """BitCol from `roots` of the DAG in order until `seconds` pass (a timing
    sample).  Returns (count, roots_completed, finished)."""
    drp, dci = _csr(drp, dci)
    n = len(drp) - 1
    r = np.ascontiguousarray(roots, dtype=np.int32)
    c = np.zeros(1, dtype=np.uint64)
    done = np.zeros(1, dtype=np.int32)
    st = _load().orc_bitcol_roots_timed(n, _p(drp), _p(dci), k, L, len(r), _p(r), float(seconds), _p(c), _p(done))
    if st not in (OK, EBUDGET):
        _check(st, "bitcol_count_roots")
    return int(c[0]), int(done[0]), st == OK


def sdegree_count_roots(drp, dci, k: int, roots, seconds: float, reduce: bool = False):
    """SDegree (with the out-neighbour reduction when `reduce`) from `roots`
    of the DAG in order until `seconds` pass (a timing sample).  Returns
    (count, roots_completed, finished)."""
    drp, dci = _csr(drp, dci)
    n = len(drp) - 1
    r = np.ascontiguousarray(roots, dtype=np.int32)
    c = np.zeros(1, dtype=np.uint64)
    done = np.zeros(1, dtype=np.int32)
    st = _load().orc_sdegree_roots_timed(n, _p(drp), _p(dci), k, 1 if reduce else 0, len(r), _p(r), float(seconds),
                                         _p(c), _p(done))
    if st not in (OK, EBUDGET):
        _check(st, "sdegree_count_roots")
    return int(c[0]), int(done[0]), st == OK


def bitcol_roots(drp, dci, k: int, roots, L: int = 32):
    """BitCol from the listed roots of the DAG only; dict of per-root arrays
    (count, nodes, isect, words) in the order of `roots`."""
    drp, dci = _csr(drp, dci)
    n = len(drp) - 1
    roots = np.ascontiguousarray(roots, dtype=np.int32)
    r = max(len(roots), 1)
    u = [np.zeros(r, dtype=np.uint64) for _ in range(4)]
    _check(_load().orc_bitcol_roots(n, _p(drp), _p(dci), k, L, len(roots), _p(roots), *[_p(a) for a in u]),
           "bitcol_roots")
    return dict(zip(["count", "nodes", "isect", "words"], [a[:len(roots)] for a in u]))


def method_count(rp, ci, k: int, method: str, L: int = 32, disable: int = 0):
    """Whole SDegree ('degree'), BitCol ('color') or SDegree-on-degeneracy
    ('core') pipeline as the paper orders it ('degree_reduced' and
    'core_reduced': SDegree with the out-neighbour reduction of Sec. 7.2); `disable` skips Pre-Core (1),
    Pre-List (2) or the pruning (4).  Returns (total, prelist_count,
    per_root dict)."""
    rp, ci = _csr(rp, ci)
    n = len(rp) - 1
    m = {"degree": 0, "color": 1, "core": 2, "degree_reduced": 3, "core_reduced": 4}[method]
    c = np.zeros(1, dtype=np.uint64)
    pl = np.zeros(1, dtype=np.uint64)
    u = [np.zeros(max(n, 1), dtype=np.uint64) for _ in range(4)]
    i3 = [np.zeros(max(n, 1), dtype=np.int32) for _ in range(3)]
    e = np.zeros(max(n, 1), dtype=np.int64)
    st = _load().orc_method_count(n, _p(rp), _p(ci), k, m, L, disable, _p(c), _p(pl), *[_p(a) for a in u],
                                  *[_p(a) for a in i3], _p(e))
    _check(st, "method_count")
    d = dict(zip(["count", "nodes", "isect", "work"], [a[:n] for a in u]))
    d.update(zip(["dplus", "core", "colors"], [a[:n] for a in i3]))
    d["edges"] = e[:n]
    return int(c[0]), int(pl[0]), d
