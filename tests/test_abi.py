"""The C interface: the library builds for gfx950, loads, and exports every
function the public header declares (no GPU needed)."""
import ctypes
import os

import numpy as np
import pytest

import paper_2203_13512_amd as kc


def test_header_declares_the_boundary():
    names = kc.declared_symbols()
    for f in ["kclique_count", "kclique_list_per_vertex", "kclique_count_ex", "kclique_count_batched",
              "kclique_plan_batched", "kclique_plan_execute", "kclique_plan_destroy",
              "kc_mlp_forward", "kc_mlp_train_step", "kc_status_string", "kc_options_init",
              "kclique_workspace_size", "kc_mlp_workspace_size", "kclique_list", "kclique_count_noalloc"]:
        assert f in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(kc.LIB_PATH), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(kc.LIB_PATH)
    for name in kc.declared_symbols():
        assert hasattr(lib, name), name


def test_rate_microbenchmark_library_is_built():
    """The benchmark's rate microbenchmarks live in a library of their own."""
    path = os.path.join(os.path.dirname(kc.LIB_PATH), "libkcpeaks.so")
    assert os.path.exists(path), "build the libraries first (__graft_entry__.build())"
    lib = ctypes.CDLL(path)
    assert hasattr(lib, "kcp_measure")
    assert not hasattr(lib, "kclique_count")


def test_status_strings_without_device():
    lib = kc._lib()
    for st in (0, -1, -2, -3, -4, -5, -6):
        assert lib.kc_status_string(st) and lib.kc_status_string(st) != b"unknown status"


def test_struct_layouts_match_header():
    # sizes fixed by the header's field order on x86-64
    assert ctypes.sizeof(kc.Stats) == 5 * 8 + 2 * 4 + 8 + 2 * 4 + 8 * 8 + 3 * 10 * 8
    assert kc.Options.stats.offset == ctypes.sizeof(kc.Options) - 8


def test_mlp_param_count():
    assert kc.MLP_NPARAMS == 4 * 64 + 64 + 64 * 64 + 64 + 64 + 1


def test_binding_refuses_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(kc, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(kc, "_LIB", None)
    with pytest.raises(RuntimeError):
        kc._lib()


def _header_fields(struct_name):
    import re
    text = open(kc.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    body = re.search(r"typedef struct \{((?:(?!typedef struct).)*?)\}\s*" + struct_name + r"\s*;", text,
                     flags=re.S).group(1)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        m = re.search(r"\**\s*(\w+)\s*(\[\d+\])?$", decl)
        names.append(m.group(1))
    return names


def test_binding_structs_follow_the_header_field_order():
    assert [f[0] for f in kc.Options._fields_] == _header_fields("kc_options")
    assert [f[0] for f in kc.Stats._fields_] == _header_fields("kc_stats")


def test_root_mask_needs_a_graph_on_the_device():
    """A root mask (kc_options.root_mask) is a device array; the binding
    refuses it with host graph arrays before any call reaches the library."""
    rp = np.array([0, 1, 2], dtype=np.int32)
    ci = np.array([1, 0], dtype=np.int32)
    mask = np.ones(2, dtype=np.uint8)
    with pytest.raises(ValueError):
        kc.count(rp, ci, 3, "color", root_mask=mask)
    with pytest.raises(ValueError):
        kc.list_cliques(rp, ci, 3, "color", capacity=4, root_mask=mask)
    with pytest.raises(ValueError):
        kc.workspace_size(rp, ci, 3, "color", root_mask=mask)
