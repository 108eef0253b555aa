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
              "qt_ctx_create", "qt_ctx_destroy", "qt_last_error"]:
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
