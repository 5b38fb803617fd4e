"""Host-side checks of the C ABI library (no GPU calls)."""
import os
import re

import pytest

from paper_2206_09983_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mnemonic.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mnemonic_[a-z_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared_functions()
    assert names == sorted(binding.EXPORTS)


def test_library_loads_and_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libmnemonic.so is not built (run __graft_entry__.build())")
    L = binding.load()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_error_codes_match_header():
    text = open(HEADER).read()
    codes = {int(v): k for k, v in re.findall(r"#define (MNEMONIC_E_[A-Z_]+) (-\d+)", text)}
    assert codes == binding.ERRORS


def test_struct_layouts_match_header_order():
    # field order of the binding's structures follows the header's typedefs
    text = open(HEADER).read()
    for cname, cls in (("mnemonic_graph", binding.mnemonic_graph), ("mnemonic_edges", binding.mnemonic_edges),
                       ("mnemonic_result", binding.mnemonic_result), ("mnemonic_stats", binding.mnemonic_stats),
                       ("mnemonic_query", binding.mnemonic_query)):
        body = re.search(r"typedef struct \{([^}]*)\}\s*%s;" % cname, text).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = re.findall(r"\*?\s*([a-z_]+)(?:\[\d\])?\s*[;,]", body)
        assert fields == [f for f, _ in cls._fields_], cname


def test_create_without_graph_is_an_argument_error_before_any_device_call():
    L = binding.load()
    import ctypes as C
    ctx = C.c_void_p()
    rc = L.mnemonic_create(None, None, 0, None, None, C.byref(ctx))
    assert rc == -1
    assert L.mnemonic_last_error(None).decode() != ""
