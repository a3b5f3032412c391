"""Exact k-clique counting on an AMD Instinct MI355X (gfx950).

Thin binding over the C interface in ``include/kclique.h`` (library
``libkclique.so`` next to this file).  Arguments are marshalled into the C
calls; every step of the computation runs in the library's HIP kernels.  The
binding refuses to run when the library is missing -- there is no fallback.

Graph arguments are int32 CSR arrays (symmetric, rows sorted, no loops):
either torch tensors on the GPU (used in place, on torch's current stream) or
numpy arrays on the host (copied by the library).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkclique.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "kclique.h")

OK, EINVAL, ENOMEM, EOVERFLOW, EDEVICE, EUNSUPPORTED, EWORKSPACE = 0, -1, -2, -3, -4, -5, -6
ORDERS = {"degree": 0, "color": 1, "core": 2, "degree_reduced": 3, "core_reduced": 4}
NO_PRECORE, NO_PRELIST, NO_PRUNE = 1, 2, 4
SCHEDULES = {"degree": 0, "learned": 1}
MLP_IN, MLP_HIDDEN = 4, 64
MLP_NPARAMS = MLP_IN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1


class KCliqueError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = _lib().kc_status_string(status).decode() if _LIB is not None else str(status)
        super().__init__(f"{what}: {msg} (status {status})")


class Stats(ctypes.Structure):
    _fields_ = [
        ("total_ms", ctypes.c_double), ("prep_ms", ctypes.c_double), ("stage_ms", ctypes.c_double),
        ("sched_ms", ctypes.c_double), ("list_ms", ctypes.c_double), ("list_launches", ctypes.c_int32),
        ("n_roots", ctypes.c_int32), ("n_tasks", ctypes.c_int64), ("max_out_degree", ctypes.c_int32),
        ("max_core", ctypes.c_int32), ("prelist_count", ctypes.c_uint64), ("nodes", ctypes.c_uint64),
        ("isect", ctypes.c_uint64), ("work", ctypes.c_uint64), ("staged_words", ctypes.c_uint64),
        ("stage_bytes", ctypes.c_uint64), ("isect_wide", ctypes.c_uint64), ("isect_compressed", ctypes.c_uint64),
        ("class_ms", ctypes.c_double * 10), ("class_work", ctypes.c_uint64 * 10),
        ("class_tasks", ctypes.c_int64 * 10),
    ]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if hasattr(v, "__len__") else v
        return d


class Options(ctypes.Structure):
    _fields_ = [
        ("device_ptrs", ctypes.c_int32), ("stream", ctypes.c_void_p), ("trusted_input", ctypes.c_int32),
        ("schedule", ctypes.c_int32), ("mlp_params", ctypes.c_void_p), ("mlp_norm", ctypes.c_void_p),
        ("waves_per_root", ctypes.c_int32), ("chunk", ctypes.c_int32), ("split", ctypes.c_int32),
        ("split_threshold", ctypes.c_float), ("compress", ctypes.c_int32), ("compress_level", ctypes.c_int32),
        ("class_streams", ctypes.c_int32), ("disable", ctypes.c_int32), ("split_policy", ctypes.c_int32),
        ("root_work", ctypes.c_void_p), ("root_isect", ctypes.c_void_p),
        ("root_features", ctypes.c_void_p), ("root_count", ctypes.c_void_p), ("vertex_k", ctypes.c_void_p),
        ("root_mask", ctypes.c_void_p), ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
        ("stats", ctypes.POINTER(Stats)),
    ]


_LIB = None


def _lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2203_13512_amd.build` "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)
    L.kc_status_string.restype = ctypes.c_char_p
    L.kc_status_string.argtypes = [ctypes.c_int]
    L.kclique_count.restype = ctypes.c_int
    L.kclique_count.argtypes = [i32, vp, vp, i32, i32, u64p]
    L.kclique_list_per_vertex.restype = ctypes.c_int
    L.kclique_list_per_vertex.argtypes = [i32, vp, vp, i32, i32, vp, u64p]
    L.kclique_count_ex.restype = ctypes.c_int
    L.kclique_count_ex.argtypes = [i32, vp, vp, i32, i32, ctypes.POINTER(Options), u64p, vp]
    L.kclique_count_batched.restype = ctypes.c_int
    L.kclique_count_batched.argtypes = [i32, vp, vp, vp, vp, vp, vp, i32, ctypes.POINTER(Options), vp]
    L.kclique_plan_batched.restype = ctypes.c_int
    L.kclique_plan_batched.argtypes = [i32, vp, vp, vp, vp, vp, vp, i32, ctypes.POINTER(Options),
                                       ctypes.POINTER(ctypes.c_void_p)]
    L.kclique_plan_execute.restype = ctypes.c_int
    L.kclique_plan_execute.argtypes = [vp, vp, vp]
    L.kclique_plan_destroy.restype = ctypes.c_int
    L.kclique_plan_destroy.argtypes = [vp]
    L.kc_mlp_forward.restype = ctypes.c_int
    L.kc_mlp_forward.argtypes = [vp, vp, i32, vp, vp]
    L.kc_mlp_train_step.restype = ctypes.c_int
    L.kc_mlp_train_step.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, i32, ctypes.c_float, vp, ctypes.c_size_t, vp]
    L.kc_mlp_workspace_size.restype = ctypes.c_int
    L.kc_mlp_workspace_size.argtypes = [i32, ctypes.POINTER(ctypes.c_size_t)]
    L.kclique_workspace_size.restype = ctypes.c_int
    L.kclique_workspace_size.argtypes = [i32, vp, vp, i32, i32, i32, ctypes.POINTER(Options),
                                         ctypes.POINTER(ctypes.c_size_t)]
    L.kclique_count_noalloc.restype = ctypes.c_int
    L.kclique_count_noalloc.argtypes = [i32, vp, vp, i32, i32, ctypes.POINTER(Options), u64p, vp]
    L.kclique_list.restype = ctypes.c_int
    L.kclique_list.argtypes = [i32, vp, vp, i32, i32, ctypes.POINTER(Options), vp, ctypes.c_int64,
                               ctypes.POINTER(ctypes.c_int64), u64p]
    L.kc_options_init.restype = None
    L.kc_options_init.argtypes = [ctypes.POINTER(Options)]
    _LIB = L
    return L


def declared_symbols(header: str = HEADER) -> list[str]:
    """Function names declared in the public header."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(k[c\w]*)\s*\(", text)) - {"kc_status"})


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _torch_stream(dev):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _check(st: int, what: str):
    if st != OK:
        raise KCliqueError(st, what)


_OPTION_KEYS = ("waves_per_root", "chunk", "split", "split_threshold", "compress", "compress_level",
                "class_streams", "split_policy", "disable")


def _options(schedule="degree", mlp=None, trusted=False, **launch):
    """kc_options for the keyword arguments of count(); returns (opt, keep)."""
    L = _lib()
    opt = Options()
    L.kc_options_init(ctypes.byref(opt))
    opt.trusted_input = 1 if trusted else 0
    opt.schedule = SCHEDULES[schedule]
    for key, v in launch.items():
        if key not in _OPTION_KEYS:
            raise TypeError(f"unknown option {key!r}")
        setattr(opt, key, v)
    keep = []
    if schedule == "learned":
        if mlp is None:
            raise ValueError("the learned schedule needs mlp=(params, norm) device tensors")
        params, norm = mlp
        opt.mlp_params = params.data_ptr()
        opt.mlp_norm = norm.data_ptr()
        keep += [params, norm]
    return opt, keep


def _root_mask(opt, root_mask, n, keep):
    """Sets kc_options.root_mask from a CUDA bool or uint8 tensor of n entries."""
    if root_mask is None:
        return
    import torch
    if not (_is_torch(root_mask) and root_mask.is_cuda):
        raise ValueError("root_mask must be a CUDA tensor (with the graph on the GPU)")
    if root_mask.dtype not in (torch.bool, torch.uint8) or root_mask.numel() != n:
        raise ValueError("root_mask must hold n bool or uint8 entries")
    m = root_mask.contiguous().view(torch.uint8)
    opt.root_mask = m.data_ptr()
    keep.append(m)


def _device_csr(row_ptr, col_idx):
    import torch
    rp = row_ptr.contiguous()
    ci = col_idx.contiguous()
    if rp.dtype != torch.int32 or ci.dtype != torch.int32:
        raise TypeError("row_ptr and col_idx must be int32")
    return rp, ci


def workspace_size(row_ptr, col_idx, k: int, order: str = "color", *, per_vertex: bool = False,
                   schedule: str = "degree", mlp=None, trusted: bool = False, root_mask=None, **launch) -> int:
    """Bytes of device scratch a count() with the same arguments takes from a
    caller-owned workspace (``kclique_workspace_size``: runs the call's
    preparation on the device and stops before the listing)."""
    opt, keep = _options(schedule, mlp, trusted, **launch)
    out = ctypes.c_size_t(0)
    if _is_torch(row_ptr) and row_ptr.is_cuda:
        rp, ci = _device_csr(row_ptr, col_idx)
        opt.device_ptrs = 1
        opt.stream = _torch_stream(rp.device)
        _root_mask(opt, root_mask, rp.numel() - 1, keep)
        rc = _lib().kclique_workspace_size(rp.numel() - 1, rp.data_ptr(), ci.data_ptr() if ci.numel() else None, k,
                                           ORDERS[order], 1 if per_vertex else 0, ctypes.byref(opt),
                                           ctypes.byref(out))
    else:
        if root_mask is not None:
            raise ValueError("root_mask takes a graph on the GPU")
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        rc = _lib().kclique_workspace_size(len(rp) - 1, rp.ctypes.data, ci.ctypes.data if ci.size else None, k,
                                           ORDERS[order], 1 if per_vertex else 0, ctypes.byref(opt),
                                           ctypes.byref(out))
    _check(rc, "kclique_workspace_size")
    return int(out.value)


def count(row_ptr, col_idx, k: int, order: str = "color", *, per_vertex: bool = False, schedule: str = "degree",
          mlp=None, trusted: bool = False, root_logs: bool = False, stats: bool = False, workspace=None,
          root_mask=None, **launch):
    """Number of k-cliques (and per-vertex participation).

    Returns ``count`` or, with ``per_vertex``, ``(count, pv)`` where pv[v]
    is the number of k-cliques containing v (int64 values, torch tensor on the
    GPU for GPU input, numpy array otherwise).  With ``stats`` a dict of the
    call's timings and work counters is appended; with ``root_logs`` (GPU
    input only) the per-vertex root logs (work, joins, features, cliques
    attributed to the vertex) are added to that dict.  ``workspace``: None
    (the library allocates its scratch), a CUDA uint8 tensor owned by the
    caller (at least workspace_size() bytes), or "torch" (sized with
    workspace_size() and allocated by torch for this call).  ``root_mask``
    (GPU input, k >= 3): a CUDA bool/uint8 tensor of n entries; only the
    share of the roots it marks is listed (kc_options.root_mask: results over
    masks that partition the vertices add up to the unmasked call's).  ``launch``:
    waves_per_root, chunk, split, split_threshold, compress, compress_level,
    class_streams, split_policy, disable (kc_options; none changes a result).
    """
    L = _lib()
    opt, keep = _options(schedule, mlp, trusted, **launch)
    st = Stats()
    opt.stats = ctypes.pointer(st)
    out = ctypes.c_uint64(0)
    on_gpu = _is_torch(row_ptr) and row_ptr.is_cuda
    if isinstance(workspace, str):
        if workspace != "torch":
            raise ValueError("workspace must be None, a device tensor or 'torch'")
        import torch
        nbytes = workspace_size(row_ptr, col_idx, k, order, per_vertex=per_vertex, schedule=schedule, mlp=mlp,
                                trusted=trusted, root_mask=root_mask, **launch)
        dev = row_ptr.device if on_gpu else torch.device("cuda")
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    if workspace is not None:
        opt.workspace = workspace.data_ptr()
        opt.workspace_bytes = workspace.numel() * workspace.element_size()
        keep.append(workspace)
    if on_gpu:
        import torch
        rp, ci = _device_csr(row_ptr, col_idx)
        n = rp.numel() - 1
        dev = rp.device
        opt.device_ptrs = 1
        opt.stream = _torch_stream(dev)
        _root_mask(opt, root_mask, n, keep)
        pv = torch.zeros(max(n, 1), dtype=torch.int64, device=dev) if per_vertex else None
        logs = None
        if root_logs:
            logs = dict(work=torch.zeros(max(n, 1), dtype=torch.int64, device=dev),
                        isect=torch.zeros(max(n, 1), dtype=torch.int64, device=dev),
                        features=torch.zeros((max(n, 1), 4), dtype=torch.float32, device=dev),
                        count=torch.zeros(max(n, 1), dtype=torch.int64, device=dev))
            opt.root_work = logs["work"].data_ptr()
            opt.root_isect = logs["isect"].data_ptr()
            opt.root_features = logs["features"].data_ptr()
            opt.root_count = logs["count"].data_ptr()
        rc = L.kclique_count_ex(n, rp.data_ptr(), ci.data_ptr() if ci.numel() else None, k, ORDERS[order],
                                ctypes.byref(opt), ctypes.byref(out), pv.data_ptr() if pv is not None else None)
        _check(rc, "kclique_count_ex")
        res = [int(out.value)]
        if per_vertex:
            res.append(pv[:n])
        if stats or root_logs:
            d = st.as_dict()
            if logs is not None:
                d["root_logs"] = {key: v[:n] for key, v in logs.items()}
            res.append(d)
    else:
        if root_logs or schedule == "learned" or root_mask is not None:
            raise ValueError("root logs, root masks and the learned schedule take GPU tensors")
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        n = len(rp) - 1
        pv = np.zeros(max(n, 1), dtype=np.uint64) if per_vertex else None
        rc = L.kclique_count_ex(n, rp.ctypes.data, ci.ctypes.data if ci.size else None, k, ORDERS[order],
                                ctypes.byref(opt), ctypes.byref(out), pv.ctypes.data if pv is not None else None)
        _check(rc, "kclique_count_ex")
        res = [int(out.value)]
        if per_vertex:
            res.append(pv[:n].astype(np.int64))
        if stats:
            res.append(st.as_dict())
    return res[0] if len(res) == 1 else tuple(res)


def list_cliques(row_ptr, col_idx, k: int, order: str = "color", capacity: int | None = None, *,
                 trusted: bool = False, workspace=None, root_mask=None, **launch):
    """Every k-clique (``kclique_list``): returns (rows, total), rows an
    int32 array of shape (min(total, capacity), k) of vertex ids (a torch
    tensor on the GPU for GPU input, numpy otherwise; row order and the order
    inside a row are unspecified).  Without ``capacity`` the total is counted
    first and the buffer sized to it.  ``root_mask`` as for count()."""
    L = _lib()
    if capacity is None:
        capacity = count(row_ptr, col_idx, k, order, trusted=trusted, root_mask=root_mask)
    opt, keep = _options("degree", None, trusted, **launch)
    if workspace is not None:
        opt.workspace = workspace.data_ptr()
        opt.workspace_bytes = workspace.numel() * workspace.element_size()
    written = ctypes.c_int64(0)
    total = ctypes.c_uint64(0)
    if _is_torch(row_ptr) and row_ptr.is_cuda:
        import torch
        rp, ci = _device_csr(row_ptr, col_idx)
        opt.device_ptrs = 1
        opt.stream = _torch_stream(rp.device)
        _root_mask(opt, root_mask, rp.numel() - 1, keep)
        out = torch.empty((max(capacity, 1), k), dtype=torch.int32, device=rp.device)
        rc = L.kclique_list(rp.numel() - 1, rp.data_ptr(), ci.data_ptr() if ci.numel() else None, k, ORDERS[order],
                            ctypes.byref(opt), out.data_ptr(), capacity, ctypes.byref(written), ctypes.byref(total))
    else:
        if root_mask is not None:
            raise ValueError("root_mask takes a graph on the GPU")
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        out = np.empty((max(capacity, 1), k), dtype=np.int32)
        rc = L.kclique_list(len(rp) - 1, rp.ctypes.data, ci.ctypes.data if ci.size else None, k, ORDERS[order],
                            ctypes.byref(opt), out.ctypes.data, capacity, ctypes.byref(written), ctypes.byref(total))
    _check(rc, "kclique_list")
    return out[: written.value], int(total.value)


def count_host(row_ptr, col_idx, k: int, order: str = "color") -> int:
    """The plain ``kclique_count`` entry point (host arrays)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    out = ctypes.c_uint64(0)
    _check(_lib().kclique_count(len(rp) - 1, rp.ctypes.data, ci.ctypes.data if ci.size else None, k, ORDERS[order],
                                ctypes.byref(out)), "kclique_count")
    return int(out.value)


def per_vertex_host(row_ptr, col_idx, k: int, order: str = "color"):
    """The plain ``kclique_list_per_vertex`` entry point (host arrays)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = len(rp) - 1
    pv = np.zeros(max(n, 1), dtype=np.uint64)
    out = ctypes.c_uint64(0)
    _check(_lib().kclique_list_per_vertex(n, rp.ctypes.data, ci.ctypes.data if ci.size else None, k, ORDERS[order],
                                          pv.ctypes.data, ctypes.byref(out)), "kclique_list_per_vertex")
    return int(out.value), pv[:n]


def _concat(graphs, ks):
    ns = np.asarray([len(g[0]) - 1 for g in graphs], dtype=np.int32)
    roff = np.zeros(len(graphs), dtype=np.int64)
    coff = np.zeros(len(graphs), dtype=np.int64)
    r_acc = c_acc = 0
    for i, (rp, ci) in enumerate(graphs):
        roff[i], coff[i] = r_acc, c_acc
        r_acc += len(rp)
        c_acc += len(ci)
    rp_cat = np.ascontiguousarray(np.concatenate([np.asarray(g[0], np.int32) for g in graphs]) if graphs
                                  else np.zeros(1, np.int32))
    ci_cat = np.ascontiguousarray(np.concatenate([np.asarray(g[1], np.int32) for g in graphs] + [np.zeros(1, np.int32)]))
    kk = np.ascontiguousarray(ks, dtype=np.int32)
    return ns, roff, coff, rp_cat, ci_cat, kk


def count_batched(graphs, ks, order: str = "color", **kw):
    """Counts of many graphs in one call; graphs are (row_ptr, col_idx) host
    arrays.  Returns a list of counts."""
    L = _lib()
    ns, roff, coff, rp_cat, ci_cat, kk = _concat(graphs, ks)
    out = np.zeros(max(len(graphs), 1), dtype=np.uint64)
    opt = Options()
    L.kc_options_init(ctypes.byref(opt))
    for key, v in kw.items():
        setattr(opt, key, v)
    rc = L.kclique_count_batched(len(graphs), ns.ctypes.data, roff.ctypes.data, coff.ctypes.data, rp_cat.ctypes.data,
                                 ci_cat.ctypes.data, kk.ctypes.data, ORDERS[order], ctypes.byref(opt),
                                 out.ctypes.data)
    _check(rc, "kclique_count_batched")
    return [int(x) for x in out[:len(graphs)]]


class Plan:
    """A prepared batch (``kclique_plan_batched``): ``execute()`` replays the
    captured listing phase and returns the per-graph counts; ``close()``
    releases it."""

    def __init__(self, graphs, ks, order: str = "color", **kw):
        L = _lib()
        self._h = ctypes.c_void_p(None)
        ns, roff, coff, rp_cat, ci_cat, kk = _concat(graphs, ks)
        self.n = len(graphs)
        opt = Options()
        L.kc_options_init(ctypes.byref(opt))
        keep = []
        mlp = kw.pop("mlp", None)
        if kw.get("schedule") is not None:
            kw["schedule"] = SCHEDULES[kw["schedule"]]
        if mlp is not None:
            params, norm = mlp
            opt.mlp_params, opt.mlp_norm = params.data_ptr(), norm.data_ptr()
            keep += [params, norm]
        for key, v in kw.items():
            setattr(opt, key, v)
        rc = L.kclique_plan_batched(len(graphs), ns.ctypes.data, roff.ctypes.data, coff.ctypes.data,
                                    rp_cat.ctypes.data, ci_cat.ctypes.data, kk.ctypes.data, ORDERS[order],
                                    ctypes.byref(opt), ctypes.byref(self._h))
        _check(rc, "kclique_plan_batched")

    def execute(self, stream=None):
        out = np.zeros(max(self.n, 1), dtype=np.uint64)
        _check(_lib().kclique_plan_execute(self._h, stream, out.ctypes.data), "kclique_plan_execute")
        return [int(x) for x in out[:self.n]]

    def close(self):
        if self._h:
            _lib().kclique_plan_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_batched(graphs, ks, order: str = "color", **kw) -> Plan:
    return Plan(graphs, ks, order, **kw)


# ------------------------------------------------------------------ MLP
def mlp_forward(params, x):
    """y = MLP(x) for x of shape (rows, 4); GPU tensors (float32)."""
    import torch
    rows = x.shape[0]
    y = torch.empty(rows, dtype=torch.float32, device=x.device)
    _check(_lib().kc_mlp_forward(params.data_ptr(), x.contiguous().data_ptr(), rows, y.data_ptr(),
                                 _torch_stream(x.device)), "kc_mlp_forward")
    return y


def mlp_train_step(params, x, target, m=None, v=None, t: int = 1, lr: float = 0.0, workspace=None):
    """One minibatch step; returns (loss tensor[1], grad tensor).  With lr > 0
    the parameters are updated in place by Adam using moments m, v.
    ``workspace``: None (the library allocates) or a CUDA uint8 tensor of at
    least mlp_workspace_size(rows) bytes."""
    import torch
    rows = x.shape[0]
    grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    ws, wsb = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None else (None, 0)
    _check(_lib().kc_mlp_train_step(params.data_ptr(), x.contiguous().data_ptr(), target.contiguous().data_ptr(),
                                    rows, grad.data_ptr(), loss.data_ptr(),
                                    m.data_ptr() if m is not None else None, v.data_ptr() if v is not None else None,
                                    t, lr, ws, wsb, _torch_stream(x.device)), "kc_mlp_train_step")
    return loss, grad


def mlp_workspace_size(rows: int) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib().kc_mlp_workspace_size(rows, ctypes.byref(out)), "kc_mlp_workspace_size")
    return int(out.value)
