"""Seeded synthetic graph generators (inputs only).

This package produces the synthetic workloads: simple undirected graphs as
int32 CSR arrays.  It holds none of the k-clique method's arithmetic.  The
tests and the benchmark pass its output to both the GPU library and the CPU
oracle; neither of those imports it.

The paper evaluates on ten public graphs (its dataset table) that are not
available here; these generators stand in for them at comparable scale and
structure: power-law degree distributions (Chung-Lu, R-MAT), planted cliques
and dense communities (which create the large maximum cliques and deep cores
the paper's graphs have), and an Erdos-Renyi case small enough for exhaustive
checks.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None

BASE_SEED = 2203135120


def build(force: bool = True) -> str:
    """Compiles the generator library in place with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    p32 = ctypes.POINTER(ctypes.c_int32)
    lib.gg_erdos_renyi.restype = vp
    lib.gg_erdos_renyi.argtypes = [i32, dbl, i32, p32, u64]
    lib.gg_chung_lu.restype = vp
    lib.gg_chung_lu.argtypes = [i32, dbl, dbl, dbl, i32, p32, u64]
    lib.gg_chung_lu_i0.restype = dbl
    lib.gg_chung_lu_i0.argtypes = [i32, dbl, dbl, dbl]
    lib.gg_rmat.restype = vp
    lib.gg_rmat.argtypes = [i32, i32, dbl, dbl, dbl, i32, i32, i32, dbl, u64]
    lib.gg_from_edges.restype = vp
    lib.gg_from_edges.argtypes = [i32, i64, p32, p32]
    lib.gg_status.restype = i32
    lib.gg_status.argtypes = [vp]
    lib.gg_n.restype = i32
    lib.gg_n.argtypes = [vp]
    lib.gg_nnz.restype = i64
    lib.gg_nnz.argtypes = [vp]
    lib.gg_copy.restype = None
    lib.gg_copy.argtypes = [vp, p32, p32]
    lib.gg_free.restype = None
    lib.gg_free.argtypes = [vp]
    lib.gg_stream.restype = None
    lib.gg_stream.argtypes = [u64, u64, i64, ctypes.POINTER(ctypes.c_uint64)]
    lib.gg_stream_seed.restype = u64
    lib.gg_stream_seed.argtypes = [u64, u64]
    _lib = lib
    return lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _take(handle) -> tuple[np.ndarray, np.ndarray]:
    lib = _load()
    try:
        st = lib.gg_status(handle)
        if st != 0:
            raise RuntimeError(f"graph generator failed with status {st}")
        n = lib.gg_n(handle)
        nnz = lib.gg_nnz(handle)
        rp = np.empty(n + 1, dtype=np.int32)
        ci = np.empty(max(nnz, 1), dtype=np.int32)
        lib.gg_copy(handle, _p32(rp), _p32(ci))
        return rp, np.ascontiguousarray(ci[:nnz])
    finally:
        lib.gg_free(handle)


def _sizes(sizes) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(list(sizes) if sizes else [0], dtype=np.int32))


def erdos_renyi(n: int, p: float, planted=(), seed: int = BASE_SEED):
    s = _sizes(planted)
    return _take(_load().gg_erdos_renyi(n, p, len(planted), _p32(s), seed))


def chung_lu(n: int, avg_deg: float, gamma: float, w_max: float, planted=(), seed: int = BASE_SEED):
    s = _sizes(planted)
    return _take(_load().gg_chung_lu(n, avg_deg, gamma, w_max, len(planted), _p32(s), seed))


def chung_lu_i0(n: int, avg_deg: float, gamma: float, w_max: float) -> float:
    return _load().gg_chung_lu_i0(n, avg_deg, gamma, w_max)


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, n_comm: int = 0, comm_min: int = 30,
         comm_max: int = 80, comm_p: float = 0.9, seed: int = BASE_SEED):
    return _take(_load().gg_rmat(scale, edge_factor, a, b, c, n_comm, comm_min, comm_max, comm_p, seed))


def from_edges(n: int, edges) -> tuple[np.ndarray, np.ndarray]:
    """Canonical CSR (symmetric, sorted, no loops/duplicates) from (u, v) pairs."""
    e = np.asarray(list(edges) if not isinstance(edges, np.ndarray) else edges, dtype=np.int32).reshape(-1, 2)
    src = np.ascontiguousarray(e[:, 0])
    dst = np.ascontiguousarray(e[:, 1])
    return _take(_load().gg_from_edges(n, len(e), _p32(src), _p32(dst)))


def stream(seed: int, substream: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().gg_stream(seed, substream, count, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


def stream_seed(seed: int, substream: int) -> int:
    return int(_load().gg_stream_seed(seed, substream))


# ----------------------------------------------------------------- workloads
@dataclass
class Workload:
    name: str
    graphs: list  # list of (row_ptr, col_idx)
    ks: list  # k per graph (batched) or the k values to run (single graph)
    orders: list = field(default_factory=lambda: ["degree"])
    params: dict = field(default_factory=dict)


def workload(cfg: int, scale: float = 1.0, seed: int = BASE_SEED) -> Workload:
    """The five synthetic workloads; `scale` < 1 shrinks them for quick tests.

    1  Erdos-Renyi G(2000, 0.01) + 20 planted 12-cliques; k=4; degree order.
    2  Chung-Lu n=1e6, mean degree 20, exponent 2.1, max weight 2e4; k=5, 7.
    3  R-MAT scale 20, edge factor 16, (0.57, 0.19, 0.19, 0.05) + 500 planted
       communities of 30..80 vertices at pair probability 0.9; k=8; color order.
    4  256 Chung-Lu graphs, n log-uniform in [1e3, 5e4], exponent 2.3, mean
       degree uniform in [10, 40], max weight sqrt(n * mean degree); k
       uniform in 3..9 per graph.
    5  Chung-Lu n=4e6, mean degree 30, exponent 2.0, max weight
       sqrt(n * mean degree) + 8 planted cliques (201, 160, 128, 100, 80, 64,
       50, 40); k=8.
    """
    s = gg_seed = stream_seed(seed, 1000 + cfg)
    if cfg == 1:
        n = max(50, int(round(2000 * scale)))
        g = erdos_renyi(n, 0.01, planted=[12] * max(1, int(round(20 * scale))), seed=s)
        return Workload("er2000_p0.01_planted20x12", [g], [4], ["degree"], dict(n=n, p=0.01))
    if cfg == 2:
        n = max(1000, int(round(1_000_000 * scale)))
        wmax = 20000.0 * math.sqrt(scale) if scale < 1 else 20000.0
        g = chung_lu(n, 20.0, 2.1, wmax, seed=s)
        return Workload(f"chunglu_n{n}_d20_g2.1", [g], [5, 7], ["degree", "color"],
                        dict(n=n, avg_deg=20.0, gamma=2.1, w_max=wmax))
    if cfg == 3:
        sc = 20 if scale >= 1 else max(8, 20 + int(math.floor(math.log2(scale))))
        ncomm = max(4, int(round(500 * (2 ** sc) / (2 ** 20))))
        g = rmat(sc, 16, 0.57, 0.19, 0.19, ncomm, 30, 80, 0.9, seed=s)
        return Workload(f"rmat_s{sc}_ef16_comm{ncomm}", [g], [8], ["color"],
                        dict(scale=sc, edge_factor=16, communities=ncomm))
    if cfg == 4:
        count = 256 if scale >= 1 else max(4, int(round(256 * scale)))
        r = np.random.Generator(np.random.Philox(key=gg_seed))
        graphs, ks, meta = [], [], []
        hi = 50000 if scale >= 1 else max(1500, int(50000 * scale))
        for i in range(count):
            n = int(round(math.exp(r.uniform(math.log(1000), math.log(hi)))))
            d = float(r.uniform(10.0, 40.0))
            k = int(r.integers(3, 10))
            g = chung_lu(n, d, 2.3, math.sqrt(n * d), seed=stream_seed(s, i))
            graphs.append(g)
            ks.append(k)
            meta.append((n, d, k))
        return Workload(f"batch{count}_chunglu_g2.3", graphs, ks, ["color"], dict(graphs=meta))
    if cfg == 5:
        n = max(2000, int(round(4_000_000 * scale)))
        planted = [201, 160, 128, 100, 80, 64, 50, 40]
        if scale < 1:
            planted = [max(12, int(round(p * max(scale, 0.05) ** 0.25))) for p in planted]
        g = chung_lu(n, 30.0, 2.0, math.sqrt(n * 30.0), planted=planted, seed=s)
        return Workload(f"chunglu_n{n}_d30_g2.0_planted", [g], [8], ["color"],
                        dict(n=n, avg_deg=30.0, gamma=2.0, w_max=math.sqrt(n * 30.0), planted=planted))
    raise ValueError(f"unknown workload {cfg}")
