"""Host-side checks of the C ABI library (no GPU needed): it loads, and it
exports every function that include/kv.h and include/kvnn.h declare; the
product package does not import the oracle."""
import ctypes
import os
import re

from paper_2210_08816_amd import kv, kvnn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="kv.h", prefix="kv_"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z_0-9]+)\s*\(", text)))


def test_header_matches_binding():
    assert declared_functions() == sorted(kv.ABI_SYMBOLS)
    assert declared_functions("kvnn.h", "kvnn_") == sorted(kvnn.ABI_SYMBOLS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(kv.LIB_PATH):
        from paper_2210_08816_amd import build
        build.build()
    lib = ctypes.CDLL(kv.LIB_PATH)
    for name in declared_functions() + declared_functions("kvnn.h", "kvnn_"):
        assert hasattr(lib, name), name


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2210_08816_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", src, flags=re.M), f
                assert "oracle/" not in src, f


def test_null_context_is_rejected():
    lib = kv.load()
    assert lib.kv_layout(None, None, None) == kv.KV_EINVAL
    assert lib.kv_last_error(None)
    nn = kvnn.load()
    assert nn.kvnn_num_params(None, None) == kvnn.KVNN_EINVAL
    assert nn.kvnn_create(None, None, None) == kvnn.KVNN_EINVAL
    assert nn.kvnn_last_error(None)
