"""The C-ABI library loads on a host without a GPU and exports every entry
point include/rr.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rr.h")
LIB = os.path.join(ROOT, "paper_1806_05826_amd", "librr.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rr_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("rr_setup", "rr_solve", "rr_destroy", "rr_apply_operator", "rr_last_error"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librr.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="librr.so not built")
def test_binding_matches_header():
    import paper_1806_05826_amd as rr
    for n in declared_functions():
        assert hasattr(rr, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="librr.so not built")
def test_error_paths_without_device():
    """Argument checks happen before any device work."""
    import paper_1806_05826_amd as rr
    lib = rr._lib
    assert lib.rr_destroy(None) == rr.RR_OK
    st = lib.rr_setup(None, None, None, None)
    assert st == rr.RR_ERR_INVALID_ARG
    assert "null" in rr.rr_last_error()
    info = rr.rr_setup_info()
    assert lib.rr_get_setup_info(None, ctypes.byref(info)) == rr.RR_ERR_INVALID_ARG
    X = rr.rr_csr(0, 5, 0, None, None, None)
    h = ctypes.c_void_p()
    assert lib.rr_setup(ctypes.byref(X), None, None, ctypes.byref(h)) == rr.RR_ERR_INVALID_ARG
    # versioned options: struct_size is set on construction; 0 is rejected
    o = rr.rr_setup_opts(n_clusters=3)
    assert o.struct_size == ctypes.sizeof(rr.rr_setup_opts)
    o.struct_size = 0
    assert lib.rr_setup(ctypes.byref(X), ctypes.byref(o), None, ctypes.byref(h)) == rr.RR_ERR_INVALID_ARG
    assert "struct_size" in rr.rr_last_error()
    # a workspace setup without a workspace, and a size query without X
    assert lib.rr_setup_ws(ctypes.byref(X), None, None, 0, None, ctypes.byref(h)) == rr.RR_ERR_INVALID_ARG
    n = ctypes.c_size_t()
    assert lib.rr_setup_workspace_size(None, None, None, ctypes.byref(n)) == rr.RR_ERR_INVALID_ARG
    assert lib.rr_set_allocator(ctypes.c_void_p(1), None, None) == rr.RR_ERR_INVALID_ARG


def test_option_structs_match_the_header():
    """The binding's option structs have the header's fields in order, with
    struct_size first."""
    import paper_1806_05826_amd as rr
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    for cls in (rr.rr_setup_opts, rr.rr_solve_opts, rr.rr_mlp_train_opts):
        name = cls.__name__
        body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + ";", text).group(1)
        fields = re.findall(r"\b(\w+)\s*(?:\[\w*\])?;", body)
        assert [f for f, _ in cls._fields_] == fields, name
        assert fields[0] == "struct_size"


def test_oracle_is_not_imported_by_the_product():
    """The product package never reaches the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_1806_05826_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
