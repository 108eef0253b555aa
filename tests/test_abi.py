"""The C-ABI library loads and exports every symbol include/qtthom.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qtthom.h")
LIB = os.path.join(ROOT, "paper_2512_07811_amd", "libqtthom.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*([a-z_]+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ["tt_hadamard", "tt_mpo_apply", "tt_round", "tt_dot", "ls_iterate", "homogenize",
              "qt_ctx_create", "qt_ctx_destroy", "qt_last_error", "qt_ctx_create_with_memory",
              "qt_ctx_fixed_bytes", "qt_workspace_query", "qt_ls_workspace_query"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_every_export():
    from paper_2512_07811_amd import qtt
    assert set(qtt.EXPORTS) >= set(declared_functions())


def _host_desc(qtt, modes, cap):
    """A descriptor whose device pointers are never dereferenced (host-only calls)."""
    import numpy as np
    modes = np.asarray(modes, dtype=np.int32)
    cap = np.asarray(cap, dtype=np.int32)
    off = np.zeros(len(modes), dtype=np.int64)
    for k in range(1, len(modes)):
        off[k] = off[k - 1] + cap[k - 1] * modes[k - 1] * cap[k]
    d = qtt.TTDesc(len(modes), 1, modes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                   cap.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                   off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 0, 16, 16)
    return d, (modes, cap, off)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_workspace_queries_are_host_only_and_sized():
    """qt_ctx_fixed_bytes and qt_workspace_query run without a device: the
    fixed head holds the 64 MiB of split-K partials, the rounding workspace
    grows with the capacities and is cut by max_rank, and a malformed
    descriptor or a null argument is refused with QT_EINVAL."""
    from paper_2512_07811_amd import qtt
    lib = qtt.load_library()
    fixed = int(lib.qt_ctx_fixed_bytes())
    assert fixed >= 64 << 20 and fixed % 256 == 0
    modes = [3] + [2] * 12
    sizes = {}
    for r in (8, 32, 64):
        cap = [1] + [min(r, 3 * 2 ** k, 2 ** (12 - k + 1)) for k in range(1, 13)] + [1]
        d, keep = _host_desc(qtt, modes, cap)
        for mr in (0, 4):
            b = ctypes.c_size_t()
            o = qtt.round_opts(1e-6, mr)
            assert lib.qt_workspace_query(ctypes.byref(d), ctypes.byref(o), ctypes.byref(b)) == 0
            assert b.value > 0 and b.value % 256 == 0
            sizes[(r, mr)] = b.value
    assert sizes[(8, 0)] < sizes[(32, 0)] < sizes[(64, 0)]
    assert sizes[(64, 4)] <= sizes[(64, 0)]
    bad, keep = _host_desc(qtt, modes, [2] + [4] * 12 + [1])   # boundary capacity 2
    b = ctypes.c_size_t()
    o = qtt.round_opts(1e-6, 0)
    assert lib.qt_workspace_query(ctypes.byref(bad), ctypes.byref(o), ctypes.byref(b)) == -1
    assert b"boundary" in lib.qt_last_error()
    assert lib.qt_workspace_query(None, ctypes.byref(o), ctypes.byref(b)) == -1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2512_07811_amd import qtt
    monkeypatch.setattr(qtt, "_lib", None)
    with pytest.raises(ImportError, match="missing"):
        qtt.load_library(str(tmp_path / "libqtthom.so"))


def test_binding_refuses_to_run_without_a_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a HIP device is present")
    from paper_2512_07811_amd import qtt
    with pytest.raises(RuntimeError, match="HIP device"):
        qtt._torch()


# an import of the oracle package, a path into it, or an attribute of it
USES_ORACLE = r"^\s*(from|import)\s+oracle\b|oracle/|\boracle\.[A-Za-z_]|import_module\(\s*['\"]oracle"


def test_product_sources_never_reach_the_oracle():
    """Nothing in the package (Python, HIP, C headers) imports, links or opens oracle/."""
    pkg = os.path.join(ROOT, "paper_2512_07811_amd")
    hits = []
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                if re.search(USES_ORACLE, src, flags=re.M):
                    hits.append(f)
    if re.search(USES_ORACLE, open(HEADER).read(), flags=re.M):
        hits.append("qtthom.h")
    assert hits == []
