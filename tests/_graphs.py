"""Small graph builders and fixture readers for the tests (inputs only)."""
from __future__ import annotations

import itertools
import os

import numpy as np

import graphgen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def csr(n, edges):
    return graphgen.from_edges(n, np.asarray(list(edges), dtype=np.int32).reshape(-1, 2))


def complete(n):
    return csr(n, itertools.combinations(range(n), 2))


def multipartite(parts):
    """Complete multipartite graph K_{a_1..a_r}; returns (csr, part index)."""
    owner = []
    for i, a in enumerate(parts):
        owner += [i] * a
    n = len(owner)
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if owner[u] != owner[v]]
    return csr(n, edges), np.asarray(owner)


def disjoint_union(graphs):
    edges, off = [], 0
    for rp, ci in graphs:
        n = len(rp) - 1
        for u in range(n):
            for v in ci[rp[u]:rp[u + 1]]:
                if u < v:
                    edges.append((u + off, int(v) + off))
        off += n
    return csr(off, edges)


def edges_of(rp, ci):
    out = []
    for u in range(len(rp) - 1):
        for v in ci[rp[u]:rp[u + 1]]:
            if u < v:
                out.append((u, int(v)))
    return out


def graph_from_mask(n, mask):
    pairs = list(itertools.combinations(range(n), 2))
    return csr(n, [p for i, p in enumerate(pairs) if (mask >> i) & 1])


def paper_example_graph():
    """The reconstructed running example; returns (csr with 0-based ids, n)."""
    n = None
    edges = []
    with open(os.path.join(GOLDEN, "paper_example_graph.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            a, b = line.split()
            if a == "n":
                n = int(b)
            else:
                edges.append((int(a) - 1, int(b) - 1))
    return csr(n, edges), n


def paper_expected():
    out = {}
    with open(os.path.join(GOLDEN, "paper_examples_expected.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            out[key] = vals
    return out


def induced(rp, ci, keep):
    """Induced subgraph on vertex list `keep` (relabelled 0..len-1)."""
    idx = {int(v): i for i, v in enumerate(keep)}
    edges = []
    for v in keep:
        for w in ci[rp[v]:rp[v + 1]]:
            w = int(w)
            if w in idx and int(v) < w:
                edges.append((idx[int(v)], idx[w]))
    return csr(len(keep), edges)


def py_brute_count(rp, ci, k):
    """Direct transcription of the result's definition with itertools."""
    n = len(rp) - 1
    adj = [set(int(x) for x in ci[rp[v]:rp[v + 1]]) for v in range(n)]
    cnt = 0
    pv = [0] * n
    for S in itertools.combinations(range(n), k):
        if all(b in adj[a] for a, b in itertools.combinations(S, 2)):
            cnt += 1
            for v in S:
                pv[v] += 1
    return cnt, pv


def elementary_symmetric(a, k):
    """e_k(a_1..a_r) with Python integers."""
    e = [1] + [0] * k
    for x in a:
        for j in range(k, 0, -1):
            e[j] += e[j - 1] * x
    return e[k]


def complete_minus_edge(n, a=0, b=1):
    """K_n without the edge (a, b): C(n,k) - C(n-2,k-2) k-cliques; a and b lie
    in C(n-2,k-1) of them, every other vertex in C(n-1,k-1) - C(n-3,k-3)."""
    return csr(n, [(u, v) for u, v in itertools.combinations(range(n), 2) if {u, v} != {a, b}])


def cocktail_party(r):
    """K_{2 x r}: r pairs, every vertex adjacent to all but its partner
    (vertex 2i pairs with 2i+1); e_k(2,...,2) = 2^k C(r,k) k-cliques."""
    n = 2 * r
    return csr(n, [(u, v) for u, v in itertools.combinations(range(n), 2) if u // 2 != v // 2])


def bipartite_with_clique(a, b, m):
    """Complete bipartite K_{a,b} (left 0..a-1, right a..a+b-1) plus a clique on
    the first m right vertices.  A k-clique (k >= 3) holds at most one left
    vertex and its other vertices in the clique: a C(m,k-1) + C(m,k) of them;
    a left vertex lies in C(m,k-1), a clique vertex in a C(m-1,k-2) +
    C(m-1,k-1), any other right vertex in none."""
    left, right = range(a), range(a, a + b)
    edges = [(u, v) for u in left for v in right]
    edges += list(itertools.combinations(range(a, a + m), 2))
    return csr(a + b, edges)


_WORKLOADS = {}


def workload_cached(cfg):
    """graphgen.workload(cfg) at full size, generated once per test session."""
    if cfg not in _WORKLOADS:
        _WORKLOADS[cfg] = graphgen.workload(cfg)
    return _WORKLOADS[cfg]


def graph_sha(rp, ci):
    import hashlib
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(rp, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(ci, dtype="<i4").tobytes())
    return h.hexdigest()


def array_sha(a):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u8").tobytes()).hexdigest()
